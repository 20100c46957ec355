// Internal declarations of libfwigrad (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace fwi {

// Every array a time step touches lives in one padded layout so the stencil
// needs no bounds checks: PAD_X/PAD_Y points before and after x/y, PAD_Z0
// before z (interior rows start on a 128-byte line) and tile slack plus
// PAD_Z0 after z.  The pads are zero and never written.  Kernels address a
// padded array with 32-bit byte offsets from its allocation base, so one
// padded array holds fewer than 2^30 floats (checked on the host).
constexpr int PAD_X = 8;
constexpr int PAD_Y = 8;
constexpr int PAD_Z0 = 32;
constexpr int TILE_Z = 64;     // one wave64 along z
constexpr int TILE_ZW = 128;   // one wave64 along z, two points per lane (z rounding of padded 3D arrays)
constexpr int TILE_Y = 32;     // y rounding of padded 3D arrays (largest stencil tile height)
constexpr int TILE_Z2 = 256;   // z extent of a 2D stencil workgroup

struct Padded {
    int ndim = 0;
    int nx = 0, ny = 1, nz = 0;     // computational dims (ny = 1 in 2D)
    long px = 0, py = 0, pz = 0;    // padded dims
    long sx = 0, sy = 0;            // padded strides (z stride 1)
    long origin = 0;                // offset of interior (0,0,0)
    size_t elems() const { return (size_t)px * py * pz; }
};

Padded make_padded(int ndim, const int *comp);

// ------------------------------------------------------------------ stencil
// All field pointers are allocation bases of padded arrays.
struct StepParams {
    const float *u1;        // level k-1 (forward) or k+1 (adjoint)
    const float *u2;        // level k-2 / k+2
    float *out;             // new level; may equal u2
    const float *b;         // dt^2/m
    const float *uk;        // adjoint only: forward state u^k
    float *g;               // adjoint only: gradient accumulator
    long psx, psy;          // padded strides
    long origin;            // element offset of the interior point (0,0,0)
    int nx, ny, nz, nbl;
    float kappa;            // e = kappa * b * sum(d_axis^2)
    float inv_dt2;
    float w[9];             // a_k / h^2, k = 0..R
    long src;               // origin-relative padded offset of the source node, -1 if none
    const float *wav;       // wavelet (device)
    int step;               // wavelet sample injected by this step
    int xchunk;             // x planes per workgroup
    int rpl;                // 3D: rows per lane (tile height 8 rpl), 2 or 4
    int remap;              // 3D tile order: 0 round robin, 1 XCD-contiguous, 2 z columns per XCD
    int deep;               // 3D: two planes of loads in flight (2 rows per lane)
    int vz;                 // 3D: z points per lane, 1 (64-point z tiles) or 2 (128-point tiles, 8-byte accesses)
    // forward only: sample u1 at the receivers into grow (nullptr: skip)
    const int *rec_off;     // padded offsets from the allocation base
    int nrec;
    float *grow;
};

void launch_step(const StepParams &p, int ndim, int radius, bool adjoint,
                 hipStream_t st);

// One shot's part of a batched step launch.
struct BatchEntry {
    StepParams p;
    int first;                       // first workgroup of this shot in the launch
    int ntz, nty, nwg, launched;     // tile counts (3D: launched = nwg rounded to 8)
};
// tile counts of e.p (3D uses e.p.rpl); returns the workgroups the shot
// needs, receiver-sampling workgroups included
int step_geometry(BatchEntry &e, int ndim, bool adjoint);
// tab: device array of nshot entries with increasing `first` (host_tab: the
// same entries on the host); total = the last entry's first + its
// workgroups.  3D batches use 2 rows per lane.
void launch_step_batch(const BatchEntry *tab, const BatchEntry *host_tab, int nshot, int total, int ndim,
                       int radius, bool adjoint, hipStream_t st);

// unpadded computational grid <-> padded layout
struct PadMap {
    long nx, ny, nz;        // computational dims (ny = 1 in 2D)
    long sx, sy;            // padded strides
    long origin;
};
void launch_coef(const float *m, float *b_padded, const PadMap &pm, double dt, hipStream_t st);
void launch_unpad(const float *acc_padded, float *g, const PadMap &pm, hipStream_t st);
void launch_pad(const float *f, float *dst_padded, const PadMap &pm, hipStream_t st);
// dst[(o0 + x) d0 + (o1 + y) d1 + o2 + z] += acc at computational point
// (r0 + x, r1 + y, r2 + z), over an n0 x n1 x n2 region of a padded
// accumulator (2D: index 1 unused); every target point of one launch is
// touched once, so launches issued in a fixed order sum deterministically
struct StackMap {
    PadMap pm;              // the accumulator's padded layout
    long r[3];              // region start in the computational grid
    long n[3];              // region dims
    long o[3];              // target offset
    long d0, d1;            // target strides (z contiguous)
};
void launch_stack_add(const float *acc_padded, float *dst, const StackMap &sm, hipStream_t st);
void launch_fill_zero(float *p, size_t n, hipStream_t st);
void launch_copy(float *dst, const float *src, size_t n, hipStream_t st);
struct ProbeArgs {
    const float *src[5];
    float *dst[2];
    size_t n;               // floats per stream (a multiple of the access width)
};
void launch_probe(const ProbeArgs &a, int nsrc, int ndst, int width_bytes, int grid, hipStream_t st);
void launch_gather(const float *field_origin, const int *rec_off, int nrec,
                   float *out_row, hipStream_t st);
void launch_residual(const float *d_sim, const float *d_obs, float *res,
                     size_t n, double *partials, int nparts, double *phi,
                     hipStream_t st);

// adjoint receiver injection at unique nodes (CSR over receivers); field
// pointers are allocation bases of padded arrays
struct InjectParams {
    float *lam;             // new adjoint level
    float *g;               // gradient accumulator (nullptr: no imaging term)
    const float *uk;        // forward state
    const float *b;
    const float *res_row;   // residual row of this step (nrec)
    const int *node_pad;    // padded offset (from the base) of unique node j
    const int *node_xyz;    // 3 ints per node (computational coords)
    const int *rec_ptr;     // CSR: receivers of node j = rec_idx[rec_ptr[j]..rec_ptr[j+1])
    const int *rec_idx;
    int nnode;
    int nx, ny, nz, nbl, ndim;
    float kappa, inv_dt2;
};
void launch_inject(const InjectParams &p, hipStream_t st);
// all shots of a batched step: dev_tab holds nshot entries on the device
void launch_inject_batch(const InjectParams *dev_tab, int nshot, int max_nodes, hipStream_t st);

// -------------------------------------------------------------------- codec
struct FieldView {
    int ndim;
    long n[3];          // (x, y, z); 2D fields are (nx, 1, nz)
    long sx, sy;        // element strides of x and y (z contiguous)
    // the field lives in the padded layout: rows start 16-byte aligned and
    // at least 3 zero-valued points follow the field on every axis, so the
    // codec may read and write whole 4^d blocks (writing zeros past the
    // field's end keeps those pads zero)
    int padded = 0;
};

struct CodecGeom {
    int ndim;
    long nb[3];
    long nblocks, nchunks, nsuper;
    int kblk, size, tp, guard;
    long table_bytes;   // super-chunk + chunk tables, 8-byte padded
    long max_chunk_words;
};
CodecGeom codec_geom(int ndim, const long n[3]);
long codec_bound(const CodecGeom &g);

// Device-side descriptor of one stored stream (pool bookkeeping).
struct StreamSlot {
    unsigned long long offset;   // byte offset in the pool
    unsigned long long bytes;    // stream bytes
    int valid;
    int pad;
};

// Encode `f` into stream bytes.  Scratch: chunk_words per chunk (u64),
// chunk_bits[nchunks] (u64), chunk_off[nchunks] (u64).  The destination is
// either fixed (dst != nullptr, capacity cap) or a slot of the pool stack
// (dst == nullptr: pool/pool_cap/slots/slot_index/prev_index).  Status flags
// go to `flags` (bit0 non-finite, bit1 capacity).
struct EncodeArgs {
    FieldView f;
    const float *src;            // field origin
    int max_waves = 0;           // > 0: at most this many waves, looping over the chunk groups
    double atol;
    unsigned long long *scratch;
    unsigned long long *chunk_bits;
    unsigned long long *chunk_off;
    unsigned char *dst;          // fixed destination or nullptr
    unsigned long long cap;
    unsigned char *pool;
    unsigned long long pool_cap;
    StreamSlot *slots;
    int slot_index;              // slot table entry written
    int prev_index;              // entry whose end is this stream's start, -1 = 0
    unsigned long long *out_bytes;   // device: stream bytes
    unsigned int *flags;
    unsigned long long *pool_high;
    unsigned long long *total_bytes; // device: running sum of stream bytes
};
void codec_encode(const EncodeArgs &a, hipStream_t st);

// message returned by fwi_last_error() on this thread
void set_last_error(const char *msg);

struct DecodeArgs {
    FieldView f;
    float *dst;                  // field origin
    int max_waves = 0;           // > 0: at most this many waves, looping over the chunk groups
    const unsigned char *stream; // fixed stream, or nullptr: pool slot
    const unsigned char *pool;
    const StreamSlot *slots;
    int slot_index;
    unsigned long long nbytes;   // fixed stream bytes
    unsigned int *flags;         // bit2: corrupt
};
void codec_decode(const DecodeArgs &a, hipStream_t st);
// waves of the single-field encode or decode kernel the device holds at
// once (its occupancy x the compute units); 0 if it cannot be queried
int codec_resident_waves(int ndim, bool encode);

// Several fields in one launch per pipeline stage (fields of one ndim; each
// with its own scratch, tables and destination).  host_jobs / dev_jobs:
// n * codec_job_bytes(encode) bytes each; with upload the job table is
// copied to dev_jobs on the stream before the launches, otherwise dev_jobs
// must already hold it when the launches run.
size_t codec_job_bytes(bool encode);
void codec_encode_batch(const EncodeArgs *args, int n, void *host_jobs, void *dev_jobs, bool upload,
                        hipStream_t st);
void codec_decode_batch(const DecodeArgs *args, int n, void *host_jobs, void *dev_jobs, bool upload,
                        hipStream_t st);

}  // namespace fwi
