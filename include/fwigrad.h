/*
 * libfwigrad -- checkpointed adjoint FWI gradient with lossily compressed
 * checkpoints, on one AMD Instinct MI355X (gfx950).
 *
 * The calls follow the paper's statement of the problem (Kukreja et al.,
 * "Lossy Checkpoint Compression in Full Waveform Inversion", Sec. 2):
 *   Eq. (1)  m u_tt - Lap u = q_s                 (acoustic wave equation)
 *   Eq. (2)  d_sim = P_r A(m)^-1 P_s^T q_s          (fwi_forward)
 *   Eq. (3)  Phi = 1/2 || d_sim - d_obs ||_2^2       (fwi_gradient, *phi)
 *   Eq. (4)  grad Phi = sum_t u[t] v_tt[t] = J^T dd  (fwi_gradient, fwi_backward)
 * with checkpointing (Sec. 1.3, Fig. 2) whose checkpoints are compressed by a
 * fixed-accuracy block codec (Sec. 1.4, Sec. 3; ckpt_compress).
 *
 * Discretisation (Sec. 3 "Reference Problem": 2nd order in time, high order
 * in space, absorbing layer of nbl points on every side):
 *   row k = 1..nt:  D u^k = (2M + Lap_h) u^{k-1} - B u^{k-2} + P_s^T q^{k-1}
 *   M = m/dt^2, D = M + eta/(2dt), B = M - eta/(2dt),
 *   eta = sigma_max * sum_axes (d_axis/nbl)^2 / vmax^2,
 *   sigma_max = 3 vmax ln(1000) / (2 nbl h),  d_axis = depth into the layer,
 *   Lap_h = central order-SO stencil per axis, zero outside the grid,
 *   d_sim[k-1][r] = u^k at receiver r,
 *   gradient g = -(1/dt^2) sum_k u^k (lam^k - 2 lam^{k+1} + lam^{k+2}),
 *   lam from the exact discrete adjoint, run backwards in time.
 *
 * Conventions
 *   - Arrays are C order, depth z last (contiguous): (x, z) in 2D, (x, y, z)
 *     in 3D.  A "computational grid" array has dims n[i] + 2*nbl.
 *   - Pointers marked [device] are HIP device memory owned by the caller;
 *     [host] are host memory owned by the caller.  The library owns only its
 *     workspaces and checkpoint pools (inside a context or a tape).
 *   - Every call is asynchronous on the stream passed in, except that host
 *     outputs (*phi, *nbytes, status codes that depend on device results)
 *     are produced after the call synchronises that stream.
 *   - Every function returns an int status; 0 is FWI_OK.  On error the
 *     outputs are undefined and fwi_last_error() describes the failure.  No
 *     C++ exception crosses this interface.
 */
#ifndef FWIGRAD_H
#define FWIGRAD_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    FWI_OK = 0,
    FWI_EINVAL = -1,      /* invalid argument (dims, order, atol, indices) */
    FWI_ENOMEM = -2,      /* device allocation failed */
    FWI_ECAPACITY = -3,   /* checkpoint pool or output buffer too small */
    FWI_ECORRUPT = -4,    /* compressed stream fails validation */
    FWI_ENONFINITE = -5,  /* NaN/Inf handed to the codec */
    FWI_EUNSTABLE = -6,   /* dt above the leapfrog stability limit */
    FWI_EHIP = -7,        /* HIP runtime error */
    FWI_ERANGE = -8       /* a value at or above atol * 2^23 reached the codec:
                             |decoded - x| <= atol cannot be guaranteed */
};

typedef struct fwi_ctx fwi_ctx;
typedef struct fwi_tape fwi_tape;

/* Grid and time discretisation [host].  n = PHYSICAL dims (n[2] unused in
 * 2D); space_order in {4, 8, 16}; nt = number of time steps; vmax = the
 * largest velocity of the model (m/s), used by the absorbing layer and by
 * the stability check dt <= 2h / (vmax sqrt(ndim S)), S the Nyquist value of
 * the 1D stencil symbol (checked on the host before any launch). */
typedef struct {
    int ndim;
    int n[3];
    double h;
    int space_order;
    int nbl;
    int nt;
    double dt;
    double vmax;
} fwi_grid;

/* One shot.  src: physical-grid node [host]; wavelet: [device] float32,
 * nt samples, sample k injected on the step k -> k+1; rec: [host] int32,
 * nrec x ndim physical-grid nodes (repeats allowed). */
typedef struct {
    int src[3];
    const float *wavelet;
    int nrec;
    const int32_t *rec;
} fwi_shot;

/* Checkpointing.  nslots = Revolve slots (each holds both leapfrog levels);
 * compress = 0 stores exact copies (the gradient then equals the store-all
 * gradient bit for bit), 1 stores each level compressed with absolute
 * tolerance atol; pool_bytes sizes the checkpoint pool of a tape
 * (fwi_forward_ckpt) or caps the part of the context's pool that
 * fwi_gradient may use; 0 = the context's pool size. */
typedef struct {
    int nslots;
    int compress;
    double atol;
    size_t pool_bytes;
} fwi_ckpt_cfg;

/* Timing and sizes of the last call on a context [host]. */
typedef struct {
    double ms_total;          /* whole call, HIP events */
    double ms_forward;        /* sum of forward-step kernels */
    double ms_adjoint;        /* sum of adjoint+imaging kernels */
    double ms_encode;         /* compress: encode + scan + pack */
    double ms_decode;
    long long n_forward;      /* forward-step launches */
    long long n_adjoint;
    long long n_encode;       /* fields compressed */
    long long n_decode;       /* fields decompressed */
    long long ckpt_bytes;     /* sum of stored checkpoint bytes */
    long long ckpt_raw_bytes; /* raw bytes those checkpoints represent */
    long long pool_high;      /* high-water mark of the pool (bytes) */
    long long graphs_captured; /* schedules captured into a hipGraph by the call */
    long long graphs_replayed; /* captured schedules the call replayed */
} fwi_stats;

/* Revolve action (see fwi_revolve_plan). */
enum { FWI_ADVANCE = 0, FWI_TAKESHOT = 1, FWI_RESTORE = 2, FWI_REVERSE = 3, FWI_FREE = 4 };
typedef struct { int op; int a; int b; } fwi_action;

/* Context: device ordinal and default checkpoint pool size.  Workspaces are
 * allocated lazily and reused.  Not thread-safe; one context per thread.
 * The 3D stencil's launch shape before any fwi_autotune call may be set
 * from the environment at creation (for experiments and tests):
 * FWI_XCHUNK (x planes per workgroup, default 16), FWI_RPL (rows per lane,
 * 2 or 4), FWI_REMAP (tile order 0-4), FWI_DEEP (two planes of loads in
 * flight, 0/1), FWI_VZ (z points per lane, 1 or 2; 2 ignores FWI_DEEP);
 * FWI_CODEC_WAVES caps the waves of the sweeps' checkpoint codec launches
 * (each wave then loops over several 64-chunk groups; the streams are the
 * same): a positive count, or a negative value for one resident round of
 * the codec kernel (its occupancy x the compute units); 0 or unset: one
 * wave per group. */
int fwi_ctx_create(fwi_ctx **ctx, int device, size_t pool_bytes);
int fwi_ctx_destroy(fwi_ctx *ctx);
/* Collect per-kernel HIP-event timings in later calls (small overhead). */
int fwi_ctx_set_timing(fwi_ctx *ctx, int on);
int fwi_ctx_stats(const fwi_ctx *ctx, fwi_stats *out);
/* Captured schedules: with on != 0, fwi_gradient, fwi_gradient_batch,
 * fwi_gradient_stack and the tape calls (fwi_forward_ckpt(_batch),
 * fwi_backward(_batch), fwi_backward_stack) record the whole checkpoint
 * schedule of a call (every step, codec and receiver launch) into a
 * hipGraph the first time a call signature (grid, shot, pointers, checkpoint
 * config, launch shapes; for tapes also the tape's buffers) is seen, and
 * replay it on later calls with the same signature; a graph is re-captured
 * after any of the library's buffers is reallocated.  A freed tape's buffers
 * are kept by its context (up to 64 tapes while graphs are on, 4 otherwise,
 * and beyond the newest one at most 16 GiB) and reused by the next tape of
 * the same sizes, preferring the buffers last
 * used for the same shots, so the tapes of an iterative loop replay.  No
 * graph depends on the caller's model, observed data, trace, adjoint source
 * or gradient buffers: the model is read before the replay, observed data
 * and adjoint sources are copied into context buffers before it, traces are
 * recorded into context buffers and copied to d_sim after it, and gradients
 * leave the context's accumulators after it, so loops that allocate new
 * tensors every iteration (autograd) replay too.  Results are identical to direct launches.
 * Per-kernel timings are not collected during replays; launch counts are.
 * Off by default; off drops every graph. */
int fwi_ctx_set_graphs(fwi_ctx *ctx, int on);
/* Codec overlap: with on != 0 (the default), fwi_gradient and the
 * single-shot tapes run the checkpoint codec of compressed schedules on a
 * second stream of the context (default priority), ordered with events
 * against the stencil steps that share its working buffers, so encodes and
 * decodes run beside the forward and adjoint steps.  Results are identical
 * either way; per-kernel timings then overlap.  Changing it drops captured
 * schedules. */
int fwi_ctx_set_overlap(fwi_ctx *ctx, int on);
/* Message of the last failure on this thread (static storage). */
const char *fwi_last_error(void);

/* Eq. (2): d_sim [device, nt x nrec] of model m [device, computational grid,
 * squared slowness s^2/m^2]. */
int fwi_forward(fwi_ctx *ctx, const fwi_grid *g, const float *m,
                const fwi_shot *shot, float *d_sim, hipStream_t stream);

/* fwi_forward that also returns the last two levels u^nt and u^{nt-1}
 * [device, computational grid, either may be NULL]: wavefield snapshots
 * for codec studies (Sec. 3 "Evolution of compressibility"). */
int fwi_forward_state(fwi_ctx *ctx, const fwi_grid *g, const float *m,
                      const fwi_shot *shot, float *d_sim, float *u_last,
                      float *u_prev, hipStream_t stream);

/* Eqs. (3)-(4): Phi [host] and grad [device, computational grid,
 * overwritten] for observed data d_obs [device, nt x nrec], with the
 * checkpointing of cfg.  Only the forward wavefield is ever compressed; the
 * adjoint runs at full precision.  FWI_ECAPACITY if the context's pool
 * cannot hold the checkpoints (retry with fewer slots). */
int fwi_gradient(fwi_ctx *ctx, const fwi_grid *g, const float *m,
                 const fwi_shot *shot, const float *d_obs,
                 const fwi_ckpt_cfg *cfg, float *grad, double *phi,
                 hipStream_t stream);

/* Time-subsampled imaging condition, the comparison baseline of Sec. 1
 * ("Approximate methods") and Sec. 4 ("Subsampling"): both sweeps keep
 * every step, but the sum of Eq. (4) runs only over the steps k (1..nt)
 * with k = phase (mod factor), each term weighted by factor.  Only those
 * forward states are kept (exact FP32 copies in the context's pool, capped
 * at pool_bytes when that is nonzero); there is no recomputation.  factor 1
 * gives fwi_gradient's exact result bit for bit.  Arguments and outputs as
 * in fwi_gradient.  FWI_EINVAL unless factor >= 1 and 0 <= phase < factor;
 * FWI_ECAPACITY if the kept states do not fit the pool. */
int fwi_gradient_subsampled(fwi_ctx *ctx, const fwi_grid *g, const float *m,
                            const fwi_shot *shot, const float *d_obs,
                            int factor, int phase, size_t pool_bytes,
                            float *grad, double *phi, hipStream_t stream);

/* Eq. (1) rows k0+1 .. k1 from a given state: u_cur holds u^k0 and u_prev
 * u^(k0-1) on entry [device, computational grid, not aliased]; on return
 * they hold u^k1 and u^(k1-1).  Restarting the forward sweep from a stored
 * (e.g. decompressed, Sec. 3 "Forward propagation") state.  d_sim [device,
 * nt x nrec, may be NULL] receives rows k0 .. k1-1 (u^(k0+1) .. u^k1 at the
 * receivers); other rows are left alone.  Spans chained from zero states
 * reproduce fwi_forward_state bit for bit.  FWI_EINVAL unless
 * 0 <= k0 <= k1 <= nt. */
int fwi_forward_span(fwi_ctx *ctx, const fwi_grid *g, const float *m,
                     const fwi_shot *shot, int k0, int k1, float *u_cur,
                     float *u_prev, float *d_sim, hipStream_t stream);

/* Eqs. (3)-(4) for nshots shots at once: shots that share ndim, space
 * order, nt and dt (grid dims, nbl, h, vmax, source and receivers may
 * differ, e.g. uneven apertures of one survey).  All shots follow one
 * checkpoint schedule; every time step is a single stencil launch over all
 * shots; checkpoints are taken per shot.  Arrays of nshots entries [host]:
 * grids, models[i] [device, shot i's computational grid], shots, d_obs[i]
 * [device, nt x nrec_i], grads[i] [device, overwritten], phis[i] [host].
 * cfg is shared; cfg.pool_bytes (0 = the context's pool size) is the total
 * for all shots, split in proportion to their field sizes.  Each shot's
 * results equal fwi_gradient's for that shot bit for bit. */
int fwi_gradient_batch(fwi_ctx *ctx, int nshots, const fwi_grid *grids,
                       const float *const *models, const fwi_shot *shots,
                       const float *const *d_obs, const fwi_ckpt_cfg *cfg,
                       float *const *grads, double *phis, hipStream_t stream);

/* Stacking (Sec. 2: the gradient of a survey is the sum of its shots'
 * gradients; Sec. 4 "Stacking"): the shots of a batched call add into one
 * gradient array grad [device, dims n, C order, z contiguous, overwritten].
 * region 0 adds each shot's whole computational-grid gradient (shots that
 * share one grid, origin all zero); region 1 adds only its physical part,
 * the absorbing layer dropped (uneven crops of one model: the physical
 * point (0,0,0) of shot i lands at origin[i*ndim .. i*ndim+ndim-1] [host]
 * of the model's physical grid; the layer's velocities are not model
 * parameters).  The sum runs in shot order, one shot at a time, in FP32,
 * so it is deterministic (bitwise repeatable).  FWI_EINVAL if a shot's
 * region falls outside dims n or ndim differs from the shots'. */
typedef struct {
    int ndim;
    int n[3];
    int region;
    const int *origin;
} fwi_stack;

/* fwi_gradient_batch whose shot gradients are stacked into grad
 * [device] as described by *stack; phis[i] [host] per shot. */
int fwi_gradient_stack(fwi_ctx *ctx, int nshots, const fwi_grid *grids,
                       const float *const *models, const fwi_shot *shots,
                       const float *const *d_obs, const fwi_ckpt_cfg *cfg,
                       const fwi_stack *stack, float *grad, double *phis,
                       hipStream_t stream);

/* Split form for automatic differentiation: the forward sweep writes d_sim
 * and keeps its checkpoints in a new tape (owns device memory until
 * fwi_tape_free); fwi_backward then runs the reverse sweep with any
 * receiver-side adjoint source dd [device, nt x nrec] and writes
 * grad = J^T dd (Eq. 4).  A tape can be back-propagated once.  The model
 * and wavelet must stay unchanged and alive until fwi_backward returns. */
int fwi_forward_ckpt(fwi_ctx *ctx, const fwi_grid *g, const float *m,
                     const fwi_shot *shot, const fwi_ckpt_cfg *cfg,
                     float *d_sim, fwi_tape **tape, hipStream_t stream);
int fwi_backward(fwi_ctx *ctx, fwi_tape *tape, const float *dd, float *grad,
                 hipStream_t stream);
int fwi_tape_free(fwi_tape *tape);
/* Split form of fwi_gradient_batch (same shot rules): one tape for all
 * shots, arrays of nshots entries [host] of device pointers.  cfg.pool_bytes
 * (0 = the context's pool size) is the total the tape allocates, split in
 * proportion to the shots' field sizes.  fwi_backward_batch writes
 * grads[i] = J_i^T dd[i]; fwi_tape_free releases the tape.  A batched tape
 * goes only to fwi_backward_batch and a single-shot tape only to
 * fwi_backward (FWI_EINVAL otherwise). */
int fwi_forward_ckpt_batch(fwi_ctx *ctx, int nshots, const fwi_grid *grids,
                           const float *const *models, const fwi_shot *shots,
                           const fwi_ckpt_cfg *cfg, float *const *d_sim,
                           fwi_tape **tape, hipStream_t stream);
int fwi_backward_batch(fwi_ctx *ctx, fwi_tape *tape, const float *const *dd,
                       float *const *grads, hipStream_t stream);

/* One stored checkpoint stream of a compressed tape: the stream of level
 * `level` (0: u^k, 1: u^(k-1), held only where the schedule restarts
 * forward propagation from the checkpoint) in slot `slot` of shot `shot`
 * (0 for a single-shot tape).  After fwi_forward_ckpt(_batch) the tape holds
 * the checkpoints of the forward sweep; each stream is the codec stream of
 * that level as stored in the pool, byte for byte what ckpt_compress writes
 * for the same field.  *nbytes [host] receives its size; with out [device,
 * cap bytes] non-NULL the stream is copied there (asynchronous on stream;
 * FWI_ECAPACITY if cap is too small).  FWI_EINVAL for an exact-checkpoint
 * tape, an empty slot or a level the checkpoint does not hold.  Reads the
 * slot table after synchronising the stream. */
int fwi_tape_stream(fwi_tape *tape, int shot, int slot, int level, void *out,
                    size_t cap, size_t *nbytes, hipStream_t stream);

/* fwi_backward_batch whose shot gradients J_i^T dd[i] are stacked into
 * grad [device] as described by *stack (see fwi_stack). */
int fwi_backward_stack(fwi_ctx *ctx, fwi_tape *tape, const float *const *dd,
                       const fwi_stack *stack, float *grad, hipStream_t stream);

/* Pool bytes [host] that the checkpoints of cfg.nslots slots on grid g can
 * take: exact checkpoints need exactly this much; for compressed ones it is
 * the worst case (every stream at ckpt_bound), so callers usually size a
 * compressed pool from an earlier call's fwi_stats.pool_high instead. */
int fwi_ckpt_pool_bytes(const fwi_grid *g, const fwi_ckpt_cfg *cfg, size_t *bytes);

/* Codec (Sec. 1.4 / Sec. 3: ZFP-style fixed accuracy).  field [device]
 * float32, C order, ndim in {2, 3}; every decoded value is within atol of
 * the input.  That bound needs every |x| below 2^(floor(log2 atol) + 23)
 * (at most atol * 2^23): a field with a larger value is refused with
 * FWI_ERANGE (so is a compressed checkpoint schedule that meets one), since
 * the 24-bit block conversion alone would lose more than atol.
 * ckpt_bound: worst-case stream bytes [host].  ckpt_compress writes the
 * stream to out [device, cap bytes] and its size to *nbytes [host] (after a
 * stream sync); FWI_ECAPACITY if cap is too small, FWI_ENONFINITE on NaN or
 * Inf input.  ckpt_decompress validates the header and tables (host copy of
 * the header) and writes field [device]. */
int ckpt_bound(int ndim, const int n[3], size_t *max_bytes);
int ckpt_compress(fwi_ctx *ctx, const float *field, int ndim, const int n[3],
                  double atol, void *out, size_t cap, size_t *nbytes,
                  hipStream_t stream);
int ckpt_decompress(fwi_ctx *ctx, const void *stream_bytes, size_t nbytes,
                    float *field, int ndim, const int n[3], hipStream_t stream);

/* ckpt_compress for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * no context; the encode workspace (chunk bit strings, lengths, tile sums,
 * counters, status flags) is a static 32 MiB device array of the library,
 * one per GPU for the life of the process, so the call allocates nothing.
 * Same arguments and stream as ckpt_compress on the current device; fields
 * whose workspace exceeds the array (about 4M values, e.g. 161^3 or 2048^2;
 * thin fields of many partial blocks fewer) are refused with FWI_EINVAL.
 * All calls on one GPU share the array: calls that overlap on one GPU race.
 * Synchronises the stream to return *nbytes and the status. */
int ckpt_compress_static(const float *field, int ndim, const int n[3], double atol,
                         void *out, size_t cap, size_t *nbytes, hipStream_t stream);

/* The codec on a field inside a larger array [device]: element (x, y, z)
 * at origin[x*sx + y*sy + z] (2D: origin[x*sx + z]; sy ignored).  The
 * stream is the same as ckpt_compress of the dense field.  padded != 0
 * declares the array layout used for checkpoints: rows start 16-byte
 * aligned and at least 3 zero-valued points follow the field along every
 * axis inside the array; the codec then reads and writes whole 4^d blocks
 * (decompression keeps those points zero).  FWI_EINVAL for strides that
 * overlap rows or leave no room for the declared padding, or a padded view
 * with misaligned rows. */
int ckpt_compress_view(fwi_ctx *ctx, const float *origin, int ndim, const int n[3],
                       long sx, long sy, int padded, double atol, void *out,
                       size_t cap, size_t *nbytes, hipStream_t stream);
int ckpt_decompress_view(fwi_ctx *ctx, const void *stream_bytes, size_t nbytes,
                         float *origin, int ndim, const int n[3], long sx, long sy,
                         int padded, hipStream_t stream);

/* The codec (Sec. 1.4 / Sec. 3) on several dense fields of one ndim at once:
 * one launch per pipeline stage for all of them, so that fields too small
 * to fill the GPU alone (a 256^3 field is 16,384 chunks, one lane each)
 * are coded at the rate of one large field.  n [host] holds 3 ints per
 * field (the dims of field i at n + 3 i, as ckpt_compress's n[3]).
 * ckpt_compress_batch: fields[i] [device] float32, out[i] [device] with
 * cap[i] bytes, nbytes[i] [host] the stream sizes on return; every stream
 * is byte for byte what ckpt_compress writes for that field.  The status
 * covers the call as a whole (FWI_ECAPACITY, FWI_ENONFINITE, FWI_ERANGE as
 * ckpt_compress: no stream is then usable).  ckpt_decompress_batch checks
 * every header as ckpt_decompress does and writes fields[i] [device].
 * nfields >= 1; the context's codec workspace grows to the fields' sum.
 * Both synchronise the stream before returning. */
int ckpt_compress_batch(fwi_ctx *ctx, int nfields, int ndim, const int *n,
                        const float *const *fields, double atol, void *const *out,
                        const size_t *cap, size_t *nbytes, hipStream_t stream);
int ckpt_decompress_batch(fwi_ctx *ctx, int nfields, int ndim, const int *n,
                          const void *const *streams, const size_t *nbytes,
                          float *const *fields, hipStream_t stream);

/* Host-only binomial checkpoint schedule reversing states N..1 with nslots
 * slots (minimal forward steps; largest optimal split).  out [host] holds up
 * to cap actions; *nactions receives the full count (FWI_ECAPACITY if it
 * exceeds cap).  *nforward [host, may be NULL] receives the number of
 * forward steps of the schedule. */
int fwi_revolve_plan(int nsteps, int nslots, fwi_action *out, int cap,
                     int *nactions, long long *nforward);

/* Autotuner: times every candidate launch shape of the stencil kernels on
 * this grid (3D, one z point per lane: x planes per workgroup in
 * {8,16,32,64} x tile order round-robin / XCD-contiguous x {2 rows per
 * lane, 4 rows per lane, 2 rows per lane with two planes of loads in
 * flight}, plus 2 rows per lane with the z tiles of each column dealt to
 * one XCD; two z points per lane: x planes in {8,16,32,64} x the three tile
 * orders x {2, 4} rows per lane, and 128 planes with 4 rows per lane;
 * 2D: x planes in {4..64}),
 * `steps` forward and `steps` adjoint launches each on the model
 * m [device], with the buffer roles alternating as in a sweep, and keeps
 * the fastest forward and adjoint shapes for later calls on a grid of the
 * same dims and order.  Every candidate is timed once; the best eight of each
 * sweep are timed three more times, interleaved; of those within 6 % of the
 * best mean, a shape with one plane of loads in flight is preferred, then
 * the z-column order, then round robin over the XCDs, then the most x planes per workgroup (fewest halo re-reads),
 * since in a sweep the checkpoint codec shares the memory system.
 * Results [host].  Synchronises the stream; the context's
 * working fields are cleared (tapes keep their own state). */
typedef struct {
    int ncand;
    int fwd_xchunk, fwd_rows_per_lane, fwd_xcd_order;   /* order: 0 round robin, 1 XCD-contiguous, 2 z columns per XCD, 3/4 groups of 2/4 columns per XCD */
    int adj_xchunk, adj_rows_per_lane, adj_xcd_order;
    double fwd_ms, adj_ms;
    int fwd_deep, adj_deep;       /* two planes of loads in flight */
    int fwd_vz, adj_vz;           /* z points per lane: 1 (64-point z tiles) or 2 (128-point tiles, 8-byte accesses) */
} fwi_tune_result;
int fwi_autotune(fwi_ctx *ctx, const fwi_grid *g, const float *m,
                 const fwi_shot *shot, int steps, fwi_tune_result *out,
                 hipStream_t stream);

/* Autotuner for batched shots: times the batched stencil launches (one
 * launch per step for all nshots shots, as fwi_gradient_batch and the
 * batched tapes run them) with x planes per workgroup in {8,16,32,64} (3D)
 * or {4,8,16,32,64} (2D), 2 rows per lane, round-robin tile order; every
 * candidate `steps` forward and `steps` adjoint launches four times,
 * interleaved, on non-zero fields.  Keeps the fastest (or the longest x
 * chunk within 3 % of it) for later batched calls on the same shots' grids
 * in the same order; single-shot calls keep their own shapes.  A batch has
 * many more workgroups than one shot, so it often prefers longer chunks
 * (fewer halo planes re-read) than fwi_autotune picks for one shot.  The
 * launches are timed alone: where the checkpoint codec runs beside them
 * (compressed sweeps of large 3D fields) the pick can be slower than the
 * shots' own shapes, so measure before relying on it there.
 * grids, models [device], shots: nshots entries as fwi_gradient_batch
 * takes them (shared ndim, space order, nt and dt).  Results [host];
 * synchronises the stream; the batch working fields are cleared. */
int fwi_autotune_batch(fwi_ctx *ctx, int nshots, const fwi_grid *grids,
                       const float *const *models, const fwi_shot *shots,
                       int steps, fwi_tune_result *out, hipStream_t stream);

/* Times one stencil launch shape on grid g the way fwi_autotune times its
 * candidates (steps forward and steps adjoint launches on non-zero fields,
 * buffer roles alternating as in a sweep, after one untimed launch), without
 * changing the context's chosen shapes.  shape [host] = {x planes per
 * workgroup, rows per lane (2 or 4), tile order (0..2), two planes of loads
 * in flight (0/1, one z point per lane only), z points per lane (1 or 2)};
 * 2D grids use only the first.  *fwd_ms, *adj_ms [host]: mean milliseconds
 * per launch.  Synchronises the stream; the context's working fields are
 * cleared. */
int fwi_time_shape(fwi_ctx *ctx, const fwi_grid *g, const float *m,
                   const fwi_shot *shot, const int shape[5], int steps,
                   double *fwd_ms, double *adj_ms, hipStream_t stream);

/* Streaming bandwidth probe (not part of the gradient path): every
 * dst[j] (j < ndst <= 2) receives the element-wise sum of the nsrc (1..5)
 * arrays src[i]; n floats per array [device, aligned to width].  Each lane
 * accesses width bytes (4, 8 or 16) at a time with non-temporal loads and
 * stores; grid = 0 gives every lane one access (the grid covers the
 * arrays), grid > 0 lets that many workgroups of 256 lanes stride over the
 * arrays.  3 sources + 1 destination is the forward
 * stencil's stream mix, 5 + 2 the adjoint's.  Measures the practical HBM
 * ceiling per access width and serves as the kernel of known traffic that
 * calibrates hardware counters.  FWI_EINVAL for other counts, widths,
 * misaligned pointers or a grid outside 0..2^20. */
int fwi_bandwidth_probe(const float *const *src, int nsrc, float *const *dst,
                        int ndst, size_t n, int width, int grid,
                        hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* FWIGRAD_H */
