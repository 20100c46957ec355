// Host runtime of libfwigrad: argument validation, workspaces, checkpoint
// pools, the Revolve action executor and the C ABI (include/fwigrad.h).
//
// One gradient (paper Fig. 1 and Fig. 2) is a walk over the action list:
//   ADVANCE a->b  forward steps (first sweep: receivers sampled, Eq. 2)
//   TAKESHOT s,k  store x_k = (u^k, u^{k-1}) in slot s (compressed: two
//                 codec streams placed on the device-side pool stack)
//   RESTORE s,k   working state <- slot s (exact copies are read in place;
//                 compressed ones are decoded, only u^k when the next action
//                 is the reverse step that needs nothing else)
//   REVERSE k     adjoint row k fused with the imaging condition (Eq. 4);
//                 the first one forms the residual and Phi (Eq. 3)
//   FREE s        pop the slot
// Everything runs asynchronously on the caller's stream; the host only
// waits at the end for Phi, the pool status and optional timings.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <tuple>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "../../include/fwigrad.h"
#include "internal.hpp"

namespace fwi {
std::vector<fwi_action> revolve_plan(int nsteps, int nslots);
long long revolve_min_steps(int nsteps, int nslots);
}

using namespace fwi;

namespace {

thread_local std::string g_err;

struct Error {
    int code;
    std::string msg;
};

#define HIPCHK(x)                                                                          \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess)                                                              \
            throw Error{FWI_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)};         \
    } while (0)

// bumped whenever any library buffer is (re)allocated: captured schedules
// embed buffer addresses and are valid only for the generation they saw
unsigned long long g_alloc_gen = 0;

template <class T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    void ensure(size_t want, bool zero = false)
    {
        if (want <= n && p) return;
        release();
        if (want == 0) want = 1;
        if (hipMalloc(&p, want * sizeof(T)) != hipSuccess) {
            p = nullptr;
            n = 0;
            (void)hipGetLastError();
            throw Error{FWI_ENOMEM, "device allocation of " + std::to_string(want * sizeof(T)) +
                                        " bytes failed"};
        }
        n = want;
        ++g_alloc_gen;
        if (zero) HIPCHK(hipMemset(p, 0, want * sizeof(T)));
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
};

// a padded array inside the field arena
struct FieldPtr {
    float *p = nullptr;
    void release() { p = nullptr; }
};

// Array i of the arena starts at i * (stride + ARENA_STAGGER), stride = its
// bytes rounded up to 2 MiB, so the same element of the streams a step
// touches does not sit at the same offset within a 2 MiB page.
constexpr size_t ARENA_ALIGN = size_t(2) << 20;
constexpr size_t ARENA_STAGGER = size_t(12) << 10;

// Device state of one shot's gradient: the six padded arrays (one arena),
// receiver tables, recorded data, residual, reduction buffers and the
// counters of its checkpoint stream stack.  A context holds one for the
// single-shot calls and one per shot for batched calls.
struct ShotBufs {
    DevBuf<char> arena;
    size_t arena_stride = 0;
    size_t padded_elems = 0;
    FieldPtr fa, fb, la, lb, coef, gacc;
    DevBuf<int> rec_off, node_pad;
    DevBuf<int> node_xyz, rec_ptr, rec_idx;
    DevBuf<float> dsim, res, obs;        // traces, residuals, observed data staged for graphs
    DevBuf<double> partials, phi;
    DevBuf<unsigned long long> misc;     // stream bytes, pool high-water, total bytes
    DevBuf<StreamSlot> slots;
    void release()
    {
        FieldPtr *arr[6] = {&fa, &fb, &la, &lb, &coef, &gacc};
        for (FieldPtr *a : arr) a->release();
        arena.release();
        padded_elems = 0;
        rec_off.release(); node_pad.release(); node_xyz.release(); rec_ptr.release();
        rec_idx.release(); dsim.release(); res.release(); obs.release(); partials.release(); phi.release();
        misc.release(); slots.release();
    }
};

// Launch tables of batched calls (step entries, codec jobs), staged in
// pinned host memory and copied to the device just before their launch.
// Every launch of a call has its own slice, and a call ends with a stream
// synchronisation, so no copy overwrites a table a queued launch reads.
struct BatchTables {
    char *host = nullptr;
    DevBuf<char> dev;
    size_t cap = 0, used = 0;
    void ensure(size_t n)
    {
        used = 0;
        if (n <= cap) return;
        release();
        if (hipHostMalloc((void **)&host, n, hipHostMallocDefault) != hipSuccess) {
            host = nullptr;
            (void)hipGetLastError();
            throw Error{FWI_ENOMEM, "pinned allocation of launch tables failed"};
        }
        dev.ensure(n);
        cap = n;
    }
    // byte offset of a new slice of `bytes` (256-byte aligned)
    size_t take(size_t bytes)
    {
        const size_t off = used;
        used = (used + bytes + 255) & ~(size_t)255;
        if (used > cap) throw Error{FWI_EINVAL, "internal: launch tables exhausted"};
        return off;
    }
    void release()
    {
        if (host) (void)hipHostFree(host);
        host = nullptr;
        dev.release();
        cap = used = 0;
    }
};

enum Kind { K_FWD = 0, K_ADJ = 1, K_ENC = 2, K_DEC = 3, K_NKIND = 4 };

// Device buffers of a freed tape, kept by its context for the next tape of
// the same sizes: a captured tape schedule embeds buffer addresses, so
// reusing them (instead of allocating afresh) lets it replay.
struct TapeStore {
    std::string tag;                                // the shots the tape was recorded for
    std::vector<size_t> sig;                        // bytes of each buffer, in order
    std::vector<std::pair<void *, size_t>> bufs;    // (pointer, element count)
    void release()
    {
        for (auto &b : bufs)
            if (b.first) (void)hipFree(b.first);
        bufs.clear();
        sig.clear();
    }
};

template <class T>
void store_put(TapeStore &s, DevBuf<T> &b)
{
    s.bufs.push_back({(void *)b.p, b.n});
    s.sig.push_back(b.n * sizeof(T));
    b.p = nullptr;
    b.n = 0;
}

template <class T>
void store_take(TapeStore &s, size_t i, DevBuf<T> &b)
{
    b.p = (T *)s.bufs[i].first;
    b.n = s.bufs[i].second;
    s.bufs[i].first = nullptr;
}

// contexts alive in this process (a tape freed after its context releases
// its buffers instead of returning them)
std::mutex g_ctx_mu;
std::set<const void *> g_live_ctx;

}  // namespace

struct fwi_ctx {
    int device = 0;
    size_t pool_default = 0;
    DevBuf<unsigned char> pool;
    // single-shot device state (fields, receivers, data, reductions)
    ShotBufs sb;
    // per-shot device state of batched calls
    std::vector<std::unique_ptr<ShotBufs>> batch;
    BatchTables btab;
    // codec scratch
    DevBuf<unsigned long long> scratch, chunk_bits, chunk_off, misc;
    DevBuf<StreamSlot> slots;
    DevBuf<unsigned int> flags;
    // timing
    bool timing = false;
    // captured schedules: one hipGraph per call signature, replayed while
    // no library buffer has been reallocated since the capture
    bool graphs = false;
    bool capturing = false;
    struct GraphEntry {
        hipGraphExec_t exec = nullptr;
        unsigned long long gen = 0;
        long long n_forward = 0, n_adjoint = 0, n_encode = 0, n_decode = 0;
        long long ckpt_raw_bytes = 0, ckpt_bytes_host = 0;
        char *tables = nullptr;            // batched launch tables of this graph
    };
    std::map<std::string, GraphEntry> gcache;
    // the legacy null stream cannot be captured: schedules of calls made on
    // it run on this stream, ordered with events
    hipStream_t gstream = nullptr;
    hipEvent_t gfence[2] = {nullptr, nullptr};
    void drop_graphs()
    {
        for (auto &kv : gcache) {
            if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
            if (kv.second.tables) (void)hipFree(kv.second.tables);
        }
        gcache.clear();
    }
    // stencil launch shape; overridden per grid by fwi_autotune
    int xchunk3 = 0;           // 3D x planes per workgroup (0: default)
    int rpl3 = 2;              // 3D rows per lane
    int remap3 = 0;            // 3D tile order: 0 round robin, 1 XCD-contiguous, 2 z columns per XCD,
                               // 3 and 4 groups of 2 and 4 columns per XCD
    int deep3 = 0;             // 3D two planes of loads in flight
    int vz3 = 1;               // 3D z points per lane (1: 64-point z tiles, 2: 128-point)
    // wave caps of the sweeps' single-field codec launches: FWI_CODEC_WAVES
    // (0 or unset: a wave per chunk group; a negative value: one resident
    // round of the kernel, queried at creation)
    int codec_waves = 0;
    int resident[2][2] = {{0, 0}, {0, 0}};   // [ndim == 3][encode]
    int codec_cap(int ndim, bool encode) const
    {
        return codec_waves >= 0 ? codec_waves : resident[ndim == 3][encode];
    }
    struct Shape {
        int xchunk, rpl, remap, deep, vz;
    };
    std::map<std::vector<int>, std::pair<Shape, Shape>> tuned;   // grid key -> (forward, adjoint)
    // fwi_autotune_batch: x planes per workgroup of the batched launches,
    // keyed by the batch's grid keys in shot order -> (forward, adjoint)
    std::map<std::vector<int>, std::pair<int, int>> tuned_batch;
    fwi_stats stats{};
    std::vector<hipEvent_t> evpool;
    size_t evused = 0;
    // codec work of compressed single-shot schedules runs on its own stream,
    // overlapped with the stencil; ordering events come from spool
    int overlap = 1;
    hipStream_t cstream = nullptr;
    std::vector<hipEvent_t> spool;
    size_t sused = 0;
    hipStream_t codec_stream()
    {
        if (!cstream) HIPCHK(hipStreamCreateWithFlags(&cstream, hipStreamNonBlocking));
        return cstream;
    }
    hipEvent_t sev()
    {
        if (sused == spool.size()) {
            hipEvent_t e;
            HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            spool.push_back(e);
        }
        return spool[sused++];
    }
    struct Iv {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Iv> ivs;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    std::map<std::pair<int, int>, std::vector<fwi_action>> plans;
    // storage of freed tapes, newest last (at most TAPE_CACHE entries, or
    // TAPE_CACHE_GRAPHS while schedules are captured: a per-shot autograd
    // loop keeps one tape per shot alive until its backward)
    static constexpr size_t TAPE_CACHE = 4, TAPE_CACHE_GRAPHS = 64;
    std::vector<TapeStore> tape_cache;
    // a cached store whose buffer sizes equal sig (removed from the cache),
    // preferring the newest one last used for the same shots (so that a
    // shot meets the buffers its captured schedule refers to), or an empty
    // store
    TapeStore take_store(const std::vector<size_t> &sig, const std::string &tag)
    {
        for (int pass = 0; pass < 2; ++pass)
            for (size_t i = tape_cache.size(); i-- > 0;)
                if (tape_cache[i].sig == sig && (pass == 1 || tape_cache[i].tag == tag)) {
                    TapeStore s = std::move(tape_cache[i]);
                    tape_cache.erase(tape_cache.begin() + (long)i);
                    return s;
                }
        return TapeStore{};
    }
    // the oldest stores go first once there are too many or they hold more
    // than TAPE_CACHE_BYTES (the newest is always kept)
    static constexpr size_t TAPE_CACHE_BYTES = size_t(16) << 30;
    void keep_store(TapeStore &&s)
    {
        tape_cache.push_back(std::move(s));
        auto held = [&] {
            size_t b = 0;
            for (const TapeStore &t : tape_cache)
                for (size_t n : t.sig) b += n;
            return b;
        };
        while (tape_cache.size() > (graphs ? TAPE_CACHE_GRAPHS : TAPE_CACHE) ||
               (tape_cache.size() > 1 && held() > TAPE_CACHE_BYTES)) {
            tape_cache.front().release();
            tape_cache.erase(tape_cache.begin());
        }
    }

    hipEvent_t ev()
    {
        if (evused == evpool.size()) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            evpool.push_back(e);
        }
        return evpool[evused++];
    }
};

struct fwi_tape {
    fwi_ctx *ctx = nullptr;
    fwi_grid grid{};
    fwi_shot shot{};
    std::vector<int32_t> rec;
    const float *m = nullptr;
    fwi_ckpt_cfg cfg{};
    std::vector<fwi_action> acts;
    std::vector<char> both, slot_both;
    size_t next = 0;
    std::string tag;                 // grids and shots (no addresses); see take_store
    DevBuf<unsigned char> pool;
    DevBuf<StreamSlot> slots;
    DevBuf<float> xcur, xprev;
    bool used = false;
    // batched tapes: one entry per shot (the single-shot members above stay
    // unused); the schedule position `next` and `acts` are shared
    struct Shot {
        fwi_grid grid{};
        fwi_shot shot{};
        std::vector<int32_t> rec;
        const float *m = nullptr;
        DevBuf<unsigned char> pool;
        size_t cap = 0;
        DevBuf<StreamSlot> slots;
        DevBuf<float> xcur, xprev;
        DevBuf<unsigned long long> misc;
        std::vector<char> slot_both;
        void release()
        {
            pool.release(); slots.release(); xcur.release(); xprev.release(); misc.release();
        }
    };
    std::vector<std::unique_ptr<Shot>> shots;
    long long fwd_bytes = 0;         // batched: checkpoint bytes the forward stored
};

namespace {

// ---------------------------------------------------------------- set-up
struct Setup {
    int ndim = 0, R = 0, nt = 0, nbl = 0;
    int comp[3] = {1, 1, 1};
    Padded pad;
    long usx = 0, usy = 0;          // strides of the unpadded computational grid
    size_t ncomp = 0;
    double dt = 0, h = 0;
    float w[9] = {0};
    float kappa = 0, inv_dt2 = 0;
    long src_pad = -1;              // origin-relative padded offset of the source
    int nrec = 0;
    std::vector<int> rec_pad;       // base-relative padded offsets of the receivers
    std::vector<int> node_pad;
    std::vector<int> node_xyz, rec_ptr, rec_idx;
};

// a_k of the central order-2M second derivative:
// a_k = 2 (-1)^{k+1} (M!)^2 / (k^2 (M-k)! (M+k)!),  a_0 = -2 sum a_k
void stencil_weights(int so, double *a)
{
    const int M = so / 2;
    auto fact = [](int n) {
        double f = 1.0;
        for (int i = 2; i <= n; ++i) f *= i;
        return f;
    };
    double sum = 0.0;
    for (int k = 1; k <= M; ++k) {
        double v = 2.0 * fact(M) * fact(M) / ((double)k * k * fact(M - k) * fact(M + k));
        a[k] = (k & 1) ? v : -v;
        sum += a[k];
    }
    a[0] = -2.0 * sum;
}

// two z points per lane with four rows per lane would spill registers at
// radius 8 (SO16): such shapes run two rows per lane
int shape_rpl(int vz, int rpl, int radius)
{
    return (vz == 2 && radius >= 8) ? 2 : rpl;
}

void validate_grid(const fwi_grid *g)
{
    if (!g) throw Error{FWI_EINVAL, "grid is null"};
    if (g->ndim != 2 && g->ndim != 3) throw Error{FWI_EINVAL, "ndim must be 2 or 3"};
    for (int d = 0; d < g->ndim; ++d)
        if (g->n[d] < 1) throw Error{FWI_EINVAL, "physical dims must be >= 1"};
    if (g->space_order != 4 && g->space_order != 8 && g->space_order != 16)
        throw Error{FWI_EINVAL, "space_order must be 4, 8 or 16"};
    if (g->nbl < 0) throw Error{FWI_EINVAL, "nbl must be >= 0"};
    if (g->nt < 1) throw Error{FWI_EINVAL, "nt must be >= 1"};
    if (!(g->h > 0) || !std::isfinite(g->h)) throw Error{FWI_EINVAL, "h must be positive"};
    if (!(g->dt > 0) || !std::isfinite(g->dt)) throw Error{FWI_EINVAL, "dt must be positive"};
    if (!(g->vmax > 0) || !std::isfinite(g->vmax)) throw Error{FWI_EINVAL, "vmax must be positive"};
    double a[9];
    stencil_weights(g->space_order, a);
    double S = -a[0];
    for (int k = 1; k <= g->space_order / 2; ++k) S -= 2.0 * a[k] * ((k & 1) ? -1.0 : 1.0);
    const double dtmax = 2.0 * g->h / (g->vmax * std::sqrt(g->ndim * S));
    if (g->dt > dtmax)
        throw Error{FWI_EUNSTABLE, "dt " + std::to_string(g->dt) + " exceeds the stability limit " +
                                       std::to_string(dtmax)};
    for (int d = 0; d < g->ndim; ++d)
        if ((long)g->n[d] + 2L * g->nbl > (1L << 30)) throw Error{FWI_EINVAL, "grid too large"};
}

Setup make_setup(const fwi_grid *g, const fwi_shot *shot, bool need_src)
{
    validate_grid(g);
    if (!shot) throw Error{FWI_EINVAL, "shot is null"};
    Setup s;
    s.ndim = g->ndim;
    s.R = g->space_order / 2;
    s.nt = g->nt;
    s.nbl = g->nbl;
    s.dt = g->dt;
    s.h = g->h;
    for (int d = 0; d < g->ndim; ++d) s.comp[d] = g->n[d] + 2 * g->nbl;
    s.pad = make_padded(g->ndim, s.comp);
    if (s.pad.elems() >= ((size_t)1 << 30))
        throw Error{FWI_EINVAL, "grid too large: a padded field must hold fewer than 2^30 points"};
    const int nx = s.pad.nx, ny = s.pad.ny, nz = s.pad.nz;
    s.ncomp = (size_t)nx * ny * nz;
    s.usx = (long)ny * nz;
    s.usy = nz;
    double a[9];
    stencil_weights(g->space_order, a);
    for (int k = 0; k <= s.R; ++k) s.w[k] = (float)(a[k] / (g->h * g->h));
    if (g->nbl > 0) {
        const double smax = 3.0 * g->vmax * std::log(1000.0) / (2.0 * g->nbl * g->h);
        s.kappa = (float)(smax / (2.0 * g->dt * g->vmax * g->vmax * (double)g->nbl * g->nbl));
    }
    s.inv_dt2 = (float)(1.0 / (g->dt * g->dt));
    auto coords = [&](const int *p, int out[3]) {
        out[0] = p[0] + g->nbl;
        out[1] = g->ndim == 3 ? p[1] + g->nbl : 0;
        out[2] = (g->ndim == 3 ? p[2] : p[1]) + g->nbl;
    };
    auto inside = [&](const int *p) {
        for (int d = 0; d < g->ndim; ++d)
            if (p[d] < 0 || p[d] >= g->n[d]) return false;
        return true;
    };
    if (need_src) {
        if (!shot->wavelet) throw Error{FWI_EINVAL, "wavelet is null"};
        if (!inside(shot->src)) throw Error{FWI_EINVAL, "source outside the physical grid"};
        int c[3];
        coords(shot->src, c);
        s.src_pad = (long)c[0] * s.pad.sx + (long)c[1] * s.pad.sy + c[2];
    }
    if (shot->nrec < 0) throw Error{FWI_EINVAL, "nrec must be >= 0"};
    if (shot->nrec > 0 && !shot->rec) throw Error{FWI_EINVAL, "receiver list is null"};
    s.nrec = shot->nrec;
    s.rec_pad.resize(s.nrec);
    std::map<long, std::vector<int>> nodes;
    for (int r = 0; r < s.nrec; ++r) {
        const int *p = shot->rec + (size_t)r * g->ndim;
        if (!inside(p)) throw Error{FWI_EINVAL, "receiver " + std::to_string(r) + " outside the physical grid"};
        int c[3];
        coords(p, c);
        s.rec_pad[r] = (int)(s.pad.origin + (long)c[0] * s.pad.sx + (long)c[1] * s.pad.sy + c[2]);
        nodes[(long)c[0] * s.usx + (long)c[1] * s.usy + c[2]].push_back(r);
    }
    s.rec_ptr.push_back(0);
    for (auto &kv : nodes) {
        const long u = kv.first;
        const int cx = (int)(u / s.usx), cy = (int)((u / s.usy) % ny), cz = (int)(u % nz);
        s.node_pad.push_back((int)(s.pad.origin + (long)cx * s.pad.sx + (long)cy * s.pad.sy + cz));
        s.node_xyz.push_back(cx);
        s.node_xyz.push_back(cy);
        s.node_xyz.push_back(cz);
        for (int r : kv.second) s.rec_idx.push_back(r);
        s.rec_ptr.push_back((int)s.rec_idx.size());
    }
    return s;
}

template <class T>
void upload(DevBuf<T> &b, const std::vector<T> &v, hipStream_t st)
{
    b.ensure(v.size());
    if (!v.empty()) HIPCHK(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
}

// point the six arrays into the arena
void carve_fields(ShotBufs *b)
{
    FieldPtr *arr[6] = {&b->fa, &b->fb, &b->la, &b->lb, &b->coef, &b->gacc};
    for (int i = 0; i < 6; ++i)
        arr[i]->p = (float *)(b->arena.p + (size_t)i * (b->arena_stride + ARENA_STAGGER));
}

void ensure_fields(ShotBufs *b, const Setup &s)
{
    const size_t pe = s.pad.elems();
    if (pe != b->padded_elems) {
        b->arena.release();
        b->padded_elems = 0;
        b->arena_stride = (pe * sizeof(float) + ARENA_ALIGN - 1) / ARENA_ALIGN * ARENA_ALIGN;
        b->arena.ensure(6 * (b->arena_stride + ARENA_STAGGER), true);
        b->padded_elems = pe;
        carve_fields(b);
    }
}

FieldView padded_view(const Setup &s)
{
    FieldView f;
    f.ndim = s.ndim;
    f.n[0] = s.pad.nx;
    f.n[1] = s.pad.ny;
    f.n[2] = s.pad.nz;
    f.sx = s.pad.sx;
    f.sy = s.ndim == 3 ? s.pad.sy : 0;
    f.padded = 1;
    return f;
}

void ensure_codec(fwi_ctx *c, const FieldView &f, int nslot_entries)
{
    CodecGeom g = codec_geom(f.ndim, f.n);
    c->scratch.ensure((size_t)g.nchunks * g.max_chunk_words);
    c->chunk_bits.ensure((size_t)g.nchunks);
    c->chunk_off.ensure((size_t)((g.nchunks + 1023) / 1024) + 2);
    c->misc.ensure(4);
    c->flags.ensure(1);
    c->sb.slots.ensure((size_t)std::max(nslot_entries, 1));
}

// ---------------------------------------------------------------- timing
struct Timer {
    fwi_ctx *c;
    hipStream_t st;
    hipEvent_t a = nullptr;
    int kind;
    Timer(fwi_ctx *c_, hipStream_t st_, int k) : c(c_), st(st_), kind(k)
    {
        if (c->timing && !c->capturing) {
            a = c->ev();
            HIPCHK(hipEventRecord(a, st));
        }
    }
    ~Timer()
    {
        if (a) {
            hipEvent_t b = c->ev();
            (void)hipEventRecord(b, st);
            c->ivs.push_back({kind, a, b});
        }
    }
};

void begin_call(fwi_ctx *c, hipStream_t st)
{
    HIPCHK(hipSetDevice(c->device));
    c->stats = fwi_stats{};
    c->ivs.clear();
    c->evused = 0;
    c->sused = 0;
    if (c->timing) {
        if (!c->t0) {
            HIPCHK(hipEventCreate(&c->t0));
            HIPCHK(hipEventCreate(&c->t1));
        }
        HIPCHK(hipEventRecord(c->t0, st));
    }
}

void end_call(fwi_ctx *c, hipStream_t st)
{
    if (!c->timing) return;
    HIPCHK(hipEventRecord(c->t1, st));
    HIPCHK(hipEventSynchronize(c->t1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, c->t0, c->t1));
    c->stats.ms_total = ms;
    double acc[K_NKIND] = {0, 0, 0, 0};
    for (auto &iv : c->ivs) {
        float t = 0;
        HIPCHK(hipEventElapsedTime(&t, iv.a, iv.b));
        acc[iv.kind] += t;
    }
    c->stats.ms_forward = acc[K_FWD];
    c->stats.ms_adjoint = acc[K_ADJ];
    c->stats.ms_encode = acc[K_ENC];
    c->stats.ms_decode = acc[K_DEC];
}

// -------------------------------------------------------------- executor
struct Exec {
    fwi_ctx *c;
    Setup S;
    hipStream_t st;
    const float *m;
    const fwi_shot *shot;
    ShotBufs *B = &c->sb;
    unsigned long long *misc = nullptr;  // counters of the stream stack (set with the pool)
    // codec scratch of this shot (batched calls); nullptr: the context's
    unsigned long long *scr = nullptr, *cbits = nullptr, *coff = nullptr;
    float *cur = nullptr, *prev = nullptr;
    bool prev_valid = true;
    int work = 0;
    float *l1 = nullptr, *l2 = nullptr;
    int reached = 0;
    float *dsim = nullptr;           // nt x nrec, recorded in the first sweep
    const float *adj_src = nullptr;  // residual or dd
    const float *d_obs = nullptr;
    bool have_src = false;
    float *grad = nullptr;
    // checkpoints
    bool compress = false;
    double atol = 0;
    unsigned char *pool = nullptr;
    size_t pool_cap = 0;
    StreamSlot *slots = nullptr;
    size_t raw_bytes = 0;            // uncompressed: bytes of one padded level
    std::vector<char> slot_both;     // slot holds both levels
    // Codec stream (compressed schedules with overlap on; nullptr: all work
    // on st).  The working buffers W0/W1 are the only memory both streams
    // touch; for each, the event after its last use on each stream orders
    // the other stream's next use (encode of u^k runs beside the next
    // forward step, decode of the next u^k beside the current adjoint step).
    hipStream_t cs = nullptr;
    // per working buffer: event after the main stream's last use, after the
    // codec's last use, and after the codec's last write (decode) into it
    hipEvent_t wmain[2] = {nullptr, nullptr}, wcodec[2] = {nullptr, nullptr}, wdec[2] = {nullptr, nullptr};

    // cur/prev/l1/l2 are allocation bases of padded arrays
    float *at_origin(float *base) const { return base + S.pad.origin; }
    float *W0() const { return B->fa.p; }
    float *W1() const { return B->fb.p; }
    bool in_w(const float *p) const { return p == W0() || p == W1(); }

    int wslot(const float *p) const { return p == W0() ? 0 : p == W1() ? 1 : -1; }
    hipStream_t cst() const { return cs ? cs : st; }
    // main stream, before it reads (writes = false) or writes buffer p: a
    // read waits for the codec's last write into p, a write for its last use
    void main_wait(const float *p, bool writes)
    {
        const int i = wslot(p);
        if (!cs || i < 0) return;
        hipEvent_t &e = writes ? wcodec[i] : wdec[i];
        if (e) {
            HIPCHK(hipStreamWaitEvent(st, e, 0));
            if (writes) wdec[i] = nullptr;
            e = nullptr;
        }
    }
    // main stream has just used the given buffers
    void main_used(const float *a, const float *b = nullptr, const float *o = nullptr)
    {
        if (!cs) return;
        hipEvent_t e = c->sev();
        HIPCHK(hipEventRecord(e, st));
        for (const float *p : {a, b, o}) {
            const int i = wslot(p);
            if (i >= 0) wmain[i] = e;
        }
    }
    // codec stream: wait for the main stream's last use of buffer p
    void codec_wait(const float *p)
    {
        const int i = wslot(p);
        if (cs && i >= 0 && wmain[i]) HIPCHK(hipStreamWaitEvent(cs, wmain[i], 0));
    }
    void codec_used(const float *p, bool wrote)
    {
        const int i = wslot(p);
        if (!cs || i < 0) return;
        hipEvent_t e = c->sev();
        HIPCHK(hipEventRecord(e, cs));
        wcodec[i] = e;
        if (wrote) wdec[i] = e;
    }
    // start of a run: the codec stream follows everything issued so far
    void fork()
    {
        wmain[0] = wmain[1] = wcodec[0] = wcodec[1] = wdec[0] = wdec[1] = nullptr;
        cs = (compress && c->overlap) ? c->codec_stream() : nullptr;
        if (!cs) return;
        hipEvent_t e = c->sev();
        HIPCHK(hipEventRecord(e, st));
        HIPCHK(hipStreamWaitEvent(cs, e, 0));
    }
    // end of a run: the main stream follows all codec work
    void join()
    {
        if (!cs) return;
        hipEvent_t e = c->sev();
        HIPCHK(hipEventRecord(e, cs));
        HIPCHK(hipStreamWaitEvent(st, e, 0));
        wmain[0] = wmain[1] = wcodec[0] = wcodec[1] = wdec[0] = wdec[1] = nullptr;
        cs = nullptr;
    }

    PadMap padmap() const
    {
        PadMap pm;
        pm.nx = S.pad.nx;
        pm.ny = S.pad.ny;
        pm.nz = S.pad.nz;
        pm.sx = S.pad.sx;
        pm.sy = S.ndim == 3 ? S.pad.sy : 0;
        pm.origin = S.pad.origin;
        return pm;
    }

    void init_fields()
    {
        launch_coef(m, B->coef.p, padmap(), S.dt, st);
        HIPCHK(hipMemsetAsync(B->fa.p, 0, B->padded_elems * sizeof(float), st));
        HIPCHK(hipMemsetAsync(B->fb.p, 0, B->padded_elems * sizeof(float), st));
        cur = W0();
        prev = W1();
        work = 0;
        upload(B->rec_off, S.rec_pad, st);
    }

    void init_adjoint()
    {
        HIPCHK(hipMemsetAsync(B->la.p, 0, B->padded_elems * sizeof(float), st));
        HIPCHK(hipMemsetAsync(B->lb.p, 0, B->padded_elems * sizeof(float), st));
        l1 = B->la.p;
        l2 = B->lb.p;
        HIPCHK(hipMemsetAsync(B->gacc.p, 0, B->padded_elems * sizeof(float), st));
        upload(B->node_pad, S.node_pad, st);
        upload(B->node_xyz, S.node_xyz, st);
        upload(B->rec_ptr, S.rec_ptr, st);
        upload(B->rec_idx, S.rec_idx, st);
    }

    std::vector<int> grid_key() const
    {
        return {S.ndim, S.pad.nx, S.pad.ny, S.pad.nz, S.R};
    }

    void apply_shape(StepParams &p, bool adjoint) const
    {
        auto it = c->tuned.find(grid_key());
        if (it == c->tuned.end()) return;
        const fwi_ctx::Shape &sh = adjoint ? it->second.second : it->second.first;
        p.xchunk = sh.xchunk;
        p.rpl = sh.rpl;
        p.remap = sh.remap;
        p.deep = sh.deep;
        p.vz = sh.vz;
        p.rpl = shape_rpl(p.vz, p.rpl, S.R);
    }

    StepParams params() const
    {
        StepParams p{};
        p.b = B->coef.p;
        p.psx = S.pad.sx;
        p.psy = S.ndim == 3 ? S.pad.sy : 0;
        p.origin = S.pad.origin;
        p.nx = S.pad.nx;
        p.ny = S.pad.ny;
        p.nz = S.pad.nz;
        p.nbl = S.nbl;
        p.kappa = S.kappa;
        p.inv_dt2 = S.inv_dt2;
        for (int k = 0; k < 9; ++k) p.w[k] = S.w[k];
        p.src = -1;
        p.rpl = c->rpl3;
        p.remap = c->remap3;
        p.deep = c->deep3;
        p.vz = c->vz3;
        p.rpl = shape_rpl(p.vz, p.rpl, S.R);
        // short x chunks: many workgroups in flight; the 2R halo planes
        // re-read per chunk come from L2
        p.xchunk = c->xchunk3 > 0 ? c->xchunk3 : 16;
        return p;
    }

    // parameters of the forward step that produces level k (out chosen so
    // the two working buffers alternate and checkpoint memory is never written)
    StepParams fwd_params(int k, bool record)
    {
        StepParams p = params();
        apply_shape(p, false);
        p.src = S.src_pad;
        p.wav = shot->wavelet;
        p.rec_off = B->rec_off.p;
        p.nrec = S.nrec;
        p.u1 = cur;
        p.u2 = prev;
        p.out = in_w(prev) ? prev : (cur == W0() ? W1() : W0());
        p.step = k - 1;
        // the launch samples the level it reads, u^{k-1}, on first visit
        p.grow = nullptr;
        if (record && k - 1 >= 1 && k - 1 > reached) {
            p.grow = dsim + (size_t)(k - 2) * S.nrec;
            reached = k - 1;
        }
        return p;
    }

    void fwd_commit(const StepParams &p)
    {
        prev = cur;
        cur = p.out;
    }

    void check_advance(int a) const
    {
        if (work != a) throw Error{FWI_EINVAL, "internal: advance from a state not held"};
        if (!prev_valid) throw Error{FWI_EINVAL, "internal: advance without the older level"};
    }

    void advance(int a, int b, bool record)
    {
        check_advance(a);
        Timer tm(c, st, K_FWD);
        for (int k = a + 1; k <= b; ++k) {
            const StepParams p = fwd_params(k, record);
            main_wait(p.u1, false);
            main_wait(p.u2, false);
            main_wait(p.out, true);
            launch_step(p, S.ndim, S.R, false, st);
            main_used(p.u1, p.u2, p.out);
            fwd_commit(p);
        }
        c->stats.n_forward += b - a;
        work = b;
    }

    // sample the working level if the first sweep has not recorded it yet
    void flush_record()
    {
        if (dsim && work >= 1 && work > reached) {
            launch_gather(cur, B->rec_off.p, S.nrec, dsim + (size_t)(work - 1) * S.nrec, st);
            reached = work;
        }
    }

    // store x_k; the older level only when the schedule will advance from it
    void takeshot_book(int slot, int k, bool both)
    {
        if (work != k) throw Error{FWI_EINVAL, "internal: takeshot of a state not held"};
        if ((int)slot_both.size() <= slot) slot_both.resize(slot + 1, 0);
        slot_both[slot] = both;
        c->stats.ckpt_raw_bytes += (long long)(both ? 2 : 1) * (long long)S.ncomp * 4;
    }

    EncodeArgs encode_args(int slot, int lev) const
    {
        EncodeArgs e{};
        e.f = padded_view(S);
        e.src = at_origin(lev == 0 ? cur : prev);
        e.max_waves = c->codec_cap(S.ndim, true);
        e.atol = atol;
        e.scratch = scr ? scr : c->scratch.p;
        e.chunk_bits = cbits ? cbits : c->chunk_bits.p;
        e.chunk_off = coff ? coff : c->chunk_off.p;
        e.dst = nullptr;
        e.pool = pool;
        e.pool_cap = pool_cap;
        e.slots = slots;
        e.slot_index = 2 * slot + lev;
        // streams are stacked: this one starts after the last stream of
        // the slot below (or after level 0 of this slot)
        e.prev_index = lev == 1 ? 2 * slot : (slot == 0 ? -1 : 2 * (slot - 1) + (slot_both[slot - 1] ? 1 : 0));
        e.out_bytes = misc + 0;
        e.pool_high = misc + 1;
        e.total_bytes = misc + 2;
        e.flags = c->flags.p;
        return e;
    }

    void takeshot(int slot, int k, bool both)
    {
        takeshot_book(slot, k, both);
        const int levels = both ? 2 : 1;
        if (!compress) {
            const size_t off = (size_t)(2 * slot) * raw_bytes;
            launch_copy((float *)(pool + off), cur, raw_bytes / sizeof(float), st);
            if (both) launch_copy((float *)(pool + off + raw_bytes), prev, raw_bytes / sizeof(float), st);
            c->stats.ckpt_bytes += (long long)levels * (long long)raw_bytes;
            c->stats.pool_high = std::max<long long>(c->stats.pool_high,
                                                     (long long)(off + (size_t)levels * raw_bytes));
            return;
        }
        for (int lev = 0; lev < levels; ++lev) {
            const float *src = lev == 0 ? cur : prev;
            codec_wait(src);
            {
                Timer tm(c, cst(), K_ENC);
                codec_encode(encode_args(slot, lev), cst());
            }
            codec_used(src, false);
            c->stats.n_encode += 1;
        }
    }

    DecodeArgs decode_args(int slot, int lev, float *target = nullptr) const
    {
        DecodeArgs d{};
        d.f = padded_view(S);
        d.dst = at_origin(target ? target : (lev == 0 ? W0() : W1()));
        d.max_waves = c->codec_cap(S.ndim, false);
        d.stream = nullptr;
        d.pool = pool;
        d.slots = slots;
        d.slot_index = 2 * slot + lev;
        d.flags = c->flags.p;
        return d;
    }

    // working state after decoding a compressed checkpoint into t0 (and the
    // other working buffer)
    void restore_commit(int k, bool only_cur, float *t0 = nullptr)
    {
        cur = t0 ? t0 : W0();
        prev = cur == W0() ? W1() : W0();
        prev_valid = !only_cur;
        work = k;
    }

    void restore(int slot, int k, bool only_cur)
    {
        if (slot < 0) {
            main_wait(W0(), true);
            main_wait(W1(), true);
            launch_fill_zero(B->fa.p, B->padded_elems, st);
            launch_fill_zero(B->fb.p, B->padded_elems, st);
            main_used(W0(), W1());
            cur = W0();
            prev = W1();
            prev_valid = true;
        } else if (!compress) {
            const size_t off = (size_t)(2 * slot) * raw_bytes;
            cur = (float *)(pool + off);
            prev = (float *)(pool + off + raw_bytes);
            prev_valid = slot < (int)slot_both.size() && slot_both[slot];
        } else {
            // u^k alone goes to the working buffer the current state is not
            // in, so the decode can run beside the adjoint step reading it
            float *t0 = only_cur ? (cur == W0() ? W1() : W0()) : W0();
            for (int lev = 0; lev < (only_cur ? 1 : 2); ++lev) {
                float *t = lev == 0 ? t0 : (t0 == W0() ? W1() : W0());
                codec_wait(t);
                {
                    Timer tm(c, cst(), K_DEC);
                    codec_decode(decode_args(slot, lev, t), cst());
                }
                codec_used(t, true);
                c->stats.n_decode += 1;
            }
            restore_commit(k, only_cur, t0);
        }
        work = k;
    }

    // residual and Phi before the first adjoint step
    void pre_reverse(int k)
    {
        if (work != k) throw Error{FWI_EINVAL, "internal: reverse without its state"};
        if (!adj_src) {
            flush_record();
            const size_t n = (size_t)S.nt * S.nrec;
            launch_residual(dsim, d_obs, B->res.p, n, B->partials.p, (int)B->partials.n, B->phi.p, st);
            adj_src = B->res.p;
        }
    }

    StepParams adj_params()
    {
        StepParams p = params();
        apply_shape(p, true);
        p.u1 = l1;
        p.u2 = l2;
        p.out = l2;
        p.uk = cur;
        p.g = B->gacc.p;
        return p;
    }

    // receiver residuals into the new adjoint level (and their imaging term,
    // scaled by img; img = 0: the step images nothing)
    void post_reverse(int k, float img = 1.0f)
    {
        launch_inject(inject_params(k, img), st);
        end_reverse();
    }

    InjectParams inject_params(int k, float img) const
    {
        InjectParams ip{};
        ip.lam = l2;
        ip.g = img != 0.0f ? B->gacc.p : nullptr;
        ip.uk = cur;
        ip.b = B->coef.p;
        ip.res_row = adj_src + (size_t)(k - 1) * S.nrec;
        ip.node_pad = B->node_pad.p;
        ip.node_xyz = B->node_xyz.p;
        ip.rec_ptr = B->rec_ptr.p;
        ip.rec_idx = B->rec_idx.p;
        ip.nnode = (int)S.node_pad.size();
        ip.nx = S.pad.nx;
        ip.ny = S.pad.ny;
        ip.nz = S.pad.nz;
        ip.nbl = S.nbl;
        ip.ndim = S.ndim;
        ip.kappa = S.kappa;
        ip.inv_dt2 = S.inv_dt2 * img;
        return ip;
    }

    // the new adjoint level becomes the newer one
    void end_reverse()
    {
        std::swap(l1, l2);
        c->stats.n_adjoint += 1;
    }

    void reverse(int k)
    {
        pre_reverse(k);
        main_wait(cur, false);
        {
            Timer tm(c, st, K_ADJ);
            launch_step(adj_params(), S.ndim, S.R, true, st);
        }
        post_reverse(k);
        main_used(cur);
    }

    // Time-subsampled imaging: every forward step, keeping u^k (exact copy,
    // slot j at store + j raw) at the steps k = phase (mod factor); then
    // every adjoint step, imaging only at those steps with weight factor.
    // Adjoint steps that image nothing run the forward stencil without
    // source (same update, no u^k / g streams).
    void run_subsampled(int factor, int phase, char *store, size_t raw)
    {
        size_t j = 0;
        for (int k = 1; k <= S.nt; ++k) {
            {
                Timer tm(c, st, K_FWD);
                const StepParams p = fwd_params(k, true);
                launch_step(p, S.ndim, S.R, false, st);
                fwd_commit(p);
            }
            c->stats.n_forward += 1;
            work = k;
            if (k % factor == phase) {
                launch_copy((float *)(store + j * raw), cur, raw / sizeof(float), st);
                ++j;
            }
        }
        pre_reverse(S.nt);
        for (int k = S.nt; k >= 1; --k) {
            Timer tm(c, st, K_ADJ);
            if (k % factor == phase) {
                --j;
                cur = (float *)(store + j * raw);
                StepParams p = adj_params();
                p.inv_dt2 = S.inv_dt2 * (float)factor;
                launch_step(p, S.ndim, S.R, true, st);
                post_reverse(k, (float)factor);
            } else {
                StepParams p = params();
                apply_shape(p, false);
                p.u1 = l1;
                p.u2 = l2;
                p.out = l2;
                launch_step(p, S.ndim, S.R, false, st);
                post_reverse(k, 0.0f);
            }
        }
    }

    // run acts[from, to); stops before the first REVERSE if stop_at_reverse
    size_t run(const std::vector<fwi_action> &acts, const std::vector<char> &both, size_t from,
               bool stop_at_reverse)
    {
        fork();
        size_t i = from;
        for (; i < acts.size(); ++i) {
            const fwi_action &a = acts[i];
            switch (a.op) {
            case FWI_ADVANCE: advance(a.a, a.b, true); break;
            case FWI_TAKESHOT: takeshot(a.a, a.b, both[i] != 0); break;
            case FWI_RESTORE: {
                const bool only = compress && i + 1 < acts.size() && acts[i + 1].op == FWI_REVERSE;
                restore(a.a, a.b, only);
                break;
            }
            case FWI_REVERSE:
                if (stop_at_reverse) {
                    join();
                    flush_record();
                    return i;
                }
                reverse(a.a);
                break;
            case FWI_FREE: break;
            default: throw Error{FWI_EINVAL, "internal: bad action"};
            }
        }
        join();
        return i;
    }
};

const std::vector<fwi_action> &plan_for(fwi_ctx *c, int nt, int nslots)
{
    auto key = std::make_pair(nt, std::min(nslots, nt));
    auto it = c->plans.find(key);
    if (it == c->plans.end()) it = c->plans.emplace(key, revolve_plan(nt, nslots)).first;
    return it->second;
}

// flag each TAKESHOT whose state is later restored and advanced from (only
// those need the older leapfrog level; the others serve one reverse step)
std::vector<char> restart_flags(const std::vector<fwi_action> &acts)
{
    std::vector<char> both(acts.size(), 0);
    std::vector<size_t> open;   // action index of the takeshot in each slot
    for (size_t i = 0; i < acts.size(); ++i) {
        const fwi_action &a = acts[i];
        if (a.op == FWI_TAKESHOT) {
            if ((int)open.size() <= a.a) open.resize(a.a + 1);
            open[a.a] = i;
        } else if (a.op == FWI_RESTORE && a.a >= 0 && i + 1 < acts.size() &&
                   acts[i + 1].op == FWI_ADVANCE) {
            both[open[a.a]] = 1;
        }
    }
    return both;
}

// index of the first reverse step and, for the checkpoints the first sweep
// takes, whether each slot holds the older level (what a forward tape run
// leaves behind, derived from the action list so that a replayed capture
// needs no host work)
size_t first_sweep(const std::vector<fwi_action> &acts, const std::vector<char> &both,
                   std::vector<char> &slot_both)
{
    slot_both.clear();
    size_t i = 0;
    for (; i < acts.size() && acts[i].op != FWI_REVERSE; ++i)
        if (acts[i].op == FWI_TAKESHOT) {
            if ((int)slot_both.size() <= acts[i].a) slot_both.resize(acts[i].a + 1, 0);
            slot_both[acts[i].a] = both[i];
        }
    return i;
}

void check_cfg(const fwi_ckpt_cfg *cfg)
{
    if (!cfg) throw Error{FWI_EINVAL, "checkpoint config is null"};
    if (cfg->nslots < 0) throw Error{FWI_EINVAL, "nslots must be >= 0"};
    if (cfg->compress) {
        if (!(cfg->atol >= 2.2250738585072014e-308) || !std::isfinite(cfg->atol))
            throw Error{FWI_EINVAL, "atol must be a positive normal number"};
    }
}

int max_slot_used(const std::vector<fwi_action> &acts)
{
    int m = -1;
    for (auto &a : acts)
        if (a.op == FWI_TAKESHOT) m = std::max(m, a.a);
    return m + 1;
}

// prepare the checkpoint storage of an executor
void setup_ckpt(Exec &ex, const fwi_ckpt_cfg *cfg, unsigned char *pool, size_t cap, StreamSlot *slots,
                int nslots_used)
{
    ex.compress = cfg->compress != 0;
    ex.atol = cfg->atol;
    ex.pool = pool;
    ex.pool_cap = cap;
    ex.slots = slots;
    ex.raw_bytes = ex.B->padded_elems * sizeof(float);
    if (!ex.misc) ex.misc = ex.c->misc.p;
    if (!ex.compress && (size_t)nslots_used * 2 * ex.raw_bytes > cap)
        throw Error{FWI_ECAPACITY, "pool of " + std::to_string(cap) + " bytes cannot hold " +
                                       std::to_string(nslots_used) + " exact checkpoints"};
}

void finish_status(fwi_ctx *c, hipStream_t st)
{
    unsigned int fl = 0;
    unsigned long long misc[4] = {0, 0, 0, 0};
    HIPCHK(hipMemcpyAsync(&fl, c->flags.p, sizeof(fl), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(misc, c->misc.p, sizeof(misc), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (misc[1]) c->stats.pool_high = (long long)misc[1];
    if (misc[2]) c->stats.ckpt_bytes = (long long)misc[2];
    if (fl & 1u) throw Error{FWI_ENONFINITE, "non-finite wavefield reached the codec"};
    if (fl & 8u)
        throw Error{FWI_ERANGE, "a value at or above atol * 2^23 reached the codec: the fixed-accuracy "
                                "bound cannot hold at this atol (raise atol)"};
    if (fl & 2u) throw Error{FWI_ECAPACITY, "checkpoint pool overflow (use fewer slots or a larger pool)"};
    if (fl & 4u) throw Error{FWI_ECORRUPT, "checkpoint stream failed to decode"};
}

void reset_status(fwi_ctx *c, hipStream_t st)
{
    c->flags.ensure(1);
    c->misc.ensure(4);
    HIPCHK(hipMemsetAsync(c->flags.p, 0, sizeof(unsigned int), st));
    HIPCHK(hipMemsetAsync(c->misc.p, 0, 4 * sizeof(unsigned long long), st));
}

template <class F>
int guarded(F &&f)
{
    try {
        f();
        return FWI_OK;
    } catch (const Error &e) {
        g_err = e.msg;
        return e.code;
    } catch (const std::exception &e) {
        g_err = e.what();
        return FWI_EINVAL;
    } catch (...) {
        g_err = "unknown failure";
        return FWI_EINVAL;
    }
}

// ------------------------------------------------------------ batched shots
// Walks one action list for several shots in lock step.  Every time step is
// one launch of the batched stencil over all shots; checkpoint and
// receiver work stays per shot (each shot has its own stream stack).
// a batch's identity for its tuned launch shape: the shots' grid keys in order
static std::vector<int> batch_key(const std::vector<Exec> &ex)
{
    std::vector<int> k;
    for (const Exec &e : ex) {
        const std::vector<int> g = e.grid_key();
        k.insert(k.end(), g.begin(), g.end());
    }
    return k;
}

struct BatchExec {
    fwi_ctx *c;
    hipStream_t st;
    std::vector<Exec> &ex;
    int ndim, R;
    char *dev_base;            // device tables the launches read
    bool upload;               // copy each table before its launch (eager runs)
    std::vector<StepParams> ps;
    // codec stream and buffer ordering as in Exec; the shots move in lock
    // step, so working buffer i (W0 or W1) has the same role in every shot
    hipStream_t cs = nullptr;
    hipEvent_t wmain[2] = {nullptr, nullptr}, wcodec[2] = {nullptr, nullptr}, wdec[2] = {nullptr, nullptr};
    int bx[2] = {-1, -1};      // tuned batch x chunk (forward, adjoint); 0: the shots' own
    int batch_xchunk(bool adj)
    {
        if (bx[0] < 0) {
            bx[0] = bx[1] = 0;
            auto it = c->tuned_batch.find(batch_key(ex));
            if (it != c->tuned_batch.end()) {
                bx[0] = it->second.first;
                bx[1] = it->second.second;
            }
        }
        return bx[adj ? 1 : 0];
    }
    int wslot(const float *p) const { return ex[0].wslot(p); }
    hipStream_t cst() const { return cs ? cs : st; }
    void main_wait(int i, bool writes)
    {
        if (!cs || i < 0) return;
        hipEvent_t &e = writes ? wcodec[i] : wdec[i];
        if (e) {
            HIPCHK(hipStreamWaitEvent(st, e, 0));
            if (writes) wdec[i] = nullptr;
            e = nullptr;
        }
    }
    void main_used(int a, int b = -1, int o = -1)
    {
        if (!cs) return;
        hipEvent_t e = c->sev();
        HIPCHK(hipEventRecord(e, st));
        for (int i : {a, b, o})
            if (i >= 0) wmain[i] = e;
    }
    void codec_wait(int i)
    {
        if (cs && i >= 0 && wmain[i]) HIPCHK(hipStreamWaitEvent(cs, wmain[i], 0));
    }
    void codec_used(int i, bool wrote)
    {
        if (!cs || i < 0) return;
        hipEvent_t e = c->sev();
        HIPCHK(hipEventRecord(e, cs));
        wcodec[i] = e;
        if (wrote) wdec[i] = e;
    }
    void fork()
    {
        wmain[0] = wmain[1] = wcodec[0] = wcodec[1] = wdec[0] = wdec[1] = nullptr;
        cs = (ex[0].compress && c->overlap) ? c->codec_stream() : nullptr;
        if (!cs) return;
        hipEvent_t e = c->sev();
        HIPCHK(hipEventRecord(e, st));
        HIPCHK(hipStreamWaitEvent(cs, e, 0));
    }
    void join()
    {
        if (!cs) return;
        hipEvent_t e = c->sev();
        HIPCHK(hipEventRecord(e, cs));
        HIPCHK(hipStreamWaitEvent(st, e, 0));
        wmain[0] = wmain[1] = wcodec[0] = wcodec[1] = wdec[0] = wdec[1] = nullptr;
        cs = nullptr;
    }

    void launch(bool adj)
    {
        const int n = (int)ex.size();
        BatchTables &t = c->btab;
        const size_t off = t.take((size_t)n * sizeof(BatchEntry));
        BatchEntry *h = (BatchEntry *)(t.host + off);
        int first = 0;
        for (int i = 0; i < n; ++i) {
            h[i] = BatchEntry{};
            h[i].p = ps[i];
            h[i].p.rpl = 2;             // the batched 3D kernel uses 2 rows per lane, one z point each
            h[i].p.vz = 1;
            // and deals tiles round robin: the column orders pad every shot's
            // range to a multiple of 8 G z-columns, idle workgroups that cost
            // more across many small shots than the locality gains (32 crops
            // of the batched survey: forward 3.05-3.09 ms in order 0 against
            // 3.10-3.37 ms in orders 2-4)
            h[i].p.remap = 0;
            if (const int xc = batch_xchunk(adj)) h[i].p.xchunk = xc;
            h[i].first = first;
            // every shot starts on a multiple of 8 workgroups, so that its
            // tile order sees the XCD a workgroup runs on (hardware deals
            // workgroups to the 8 XCDs round robin); the padding is receiver
            // sampling blocks past the last receiver, which do nothing
            const int g = step_geometry(h[i], ndim, adj);
            first += ndim == 3 ? (g + 7) & ~7 : g;
        }
        BatchEntry *d = (BatchEntry *)(dev_base + off);
        if (upload) HIPCHK(hipMemcpyAsync(d, h, (size_t)n * sizeof(BatchEntry), hipMemcpyHostToDevice, st));
        launch_step_batch(d, h, n, first, ndim, R, adj, st);
    }

    void advance(int a, int b)
    {
        for (auto &e : ex) e.check_advance(a);
        Timer tm(c, st, K_FWD);
        ps.resize(ex.size());
        for (int k = a + 1; k <= b; ++k) {
            for (size_t i = 0; i < ex.size(); ++i) ps[i] = ex[i].fwd_params(k, true);
            const int u1 = wslot(ps[0].u1), u2 = wslot(ps[0].u2), o = wslot(ps[0].out);
            main_wait(u1, false);
            main_wait(u2, false);
            main_wait(o, true);
            launch(false);
            main_used(u1, u2, o);
            for (size_t i = 0; i < ex.size(); ++i) ex[i].fwd_commit(ps[i]);
        }
        for (auto &e : ex) e.work = b;
        c->stats.n_forward += (long long)(b - a) * (long long)ex.size();
    }

    void reverse(int k)
    {
        for (auto &e : ex) e.pre_reverse(k);
        ps.resize(ex.size());
        const int uk = wslot(ex[0].cur);
        main_wait(uk, false);
        {
            Timer tm(c, st, K_ADJ);
            for (size_t i = 0; i < ex.size(); ++i) ps[i] = ex[i].adj_params();
            launch(true);
        }
        // receiver residuals of every shot in one launch
        const int n = (int)ex.size();
        BatchTables &t = c->btab;
        const size_t off = t.take((size_t)n * sizeof(InjectParams));
        InjectParams *h = (InjectParams *)(t.host + off);
        int maxn = 0;
        for (int i = 0; i < n; ++i) {
            h[i] = ex[i].inject_params(k, 1.0f);
            maxn = std::max(maxn, h[i].nnode);
        }
        InjectParams *d = (InjectParams *)(dev_base + off);
        if (upload) HIPCHK(hipMemcpyAsync(d, h, (size_t)n * sizeof(InjectParams), hipMemcpyHostToDevice, st));
        launch_inject_batch(d, n, maxn, st);
        for (auto &e : ex) e.end_reverse();
        main_used(uk);
    }

    // compressed checkpoints: one encode pipeline (decode launch) per level
    // for all shots
    void takeshot(int slot, int k, bool both)
    {
        if (!ex[0].compress) {
            for (auto &e : ex) e.takeshot(slot, k, both);
            return;
        }
        for (auto &e : ex) e.takeshot_book(slot, k, both);
        const int n = (int)ex.size();
        std::vector<EncodeArgs> args(n);
        for (int lev = 0; lev < (both ? 2 : 1); ++lev) {
            const int src = wslot(lev == 0 ? ex[0].cur : ex[0].prev);
            codec_wait(src);
            {
                Timer tm(c, cst(), K_ENC);
                for (int i = 0; i < n; ++i) args[i] = ex[i].encode_args(slot, lev);
                const size_t off = c->btab.take((size_t)n * codec_job_bytes(true));
                codec_encode_batch(args.data(), n, c->btab.host + off, dev_base + off, upload, cst());
            }
            codec_used(src, false);
            c->stats.n_encode += n;
        }
    }

    void restore(int slot, int k, bool only_cur)
    {
        if (slot < 0 || !ex[0].compress) {
            if (slot < 0) {
                main_wait(0, true);
                main_wait(1, true);
            }
            for (auto &e : ex) e.restore(slot, k, only_cur);
            if (slot < 0) main_used(0, 1);
            return;
        }
        const int n = (int)ex.size();
        std::vector<DecodeArgs> args(n);
        // u^k alone goes to the working buffer the current state is not in
        const int t0 = only_cur && wslot(ex[0].cur) == 0 ? 1 : 0;
        auto wbuf = [&](int i, int w) { return w == 0 ? ex[i].W0() : ex[i].W1(); };
        for (int lev = 0; lev < (only_cur ? 1 : 2); ++lev) {
            const int t = lev == 0 ? t0 : 1 - t0;
            codec_wait(t);
            {
                Timer tm(c, cst(), K_DEC);
                for (int i = 0; i < n; ++i) args[i] = ex[i].decode_args(slot, lev, wbuf(i, t));
                const size_t off = c->btab.take((size_t)n * codec_job_bytes(false));
                codec_decode_batch(args.data(), n, c->btab.host + off, dev_base + off, upload, cst());
            }
            codec_used(t, true);
            c->stats.n_decode += n;
        }
        for (int i = 0; i < n; ++i) ex[i].restore_commit(k, only_cur, wbuf(i, t0));
    }

    // run acts[from, end); stops before the first REVERSE if stop_at_reverse
    size_t run(const std::vector<fwi_action> &acts, const std::vector<char> &both, size_t from = 0,
               bool stop_at_reverse = false)
    {
        fork();
        size_t i = from;
        for (; i < acts.size(); ++i) {
            const fwi_action &a = acts[i];
            switch (a.op) {
            case FWI_ADVANCE: advance(a.a, a.b); break;
            case FWI_TAKESHOT: takeshot(a.a, a.b, both[i] != 0); break;
            case FWI_RESTORE: {
                const bool only = ex[0].compress && i + 1 < acts.size() && acts[i + 1].op == FWI_REVERSE;
                restore(a.a, a.b, only);
                break;
            }
            case FWI_REVERSE:
                if (stop_at_reverse) {
                    join();
                    for (auto &e : ex) e.flush_record();
                    return i;
                }
                reverse(a.a);
                break;
            case FWI_FREE: break;
            default: throw Error{FWI_EINVAL, "internal: bad action"};
            }
        }
        join();
        return i;
    }
};

// table bytes one batched action list needs (an upper bound: every step
// launch, and two levels per checkpoint taken or restored)
size_t table_bytes_of(const std::vector<fwi_action> &acts, size_t nshots)
{
    auto slice = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t step = slice(nshots * sizeof(BatchEntry));
    const size_t inj = slice(nshots * sizeof(InjectParams));
    const size_t enc = 2 * slice(nshots * codec_job_bytes(true));
    const size_t dec = 2 * slice(nshots * codec_job_bytes(false));
    size_t n = 0;
    for (auto &a : acts) {
        if (a.op == FWI_ADVANCE) n += (size_t)(a.b - a.a) * step;
        else if (a.op == FWI_REVERSE) n += step + inj;
        else if (a.op == FWI_TAKESHOT) n += enc;
        else if (a.op == FWI_RESTORE) n += dec;
    }
    return n + 256;
}

// ------------------------------------------------------- captured schedules
struct KeyBuilder {
    std::string s;
    template <class T>
    KeyBuilder &add(const T &v)
    {
        s.append((const char *)&v, sizeof(T));
        return *this;
    }
    KeyBuilder &bytes(const void *p, size_t n)
    {
        unsigned long long h = 1469598103934665603ull;     // FNV-1a
        for (size_t i = 0; i < n; ++i) h = (h ^ ((const unsigned char *)p)[i]) * 1099511628211ull;
        return add(h).add(n);
    }
};

void key_shot(KeyBuilder &k, fwi_ctx *c, const fwi_grid *g, const fwi_shot *sh, const Setup &S)
{
    k.add(g->ndim).add(g->n).add(g->h).add(g->space_order).add(g->nbl).add(g->nt).add(g->dt).add(g->vmax);
    k.add(sh->src).add(sh->wavelet).add(sh->nrec);
    k.bytes(sh->rec, sizeof(int32_t) * (size_t)sh->nrec * (size_t)g->ndim);
    auto it = c->tuned.find({S.ndim, S.pad.nx, S.pad.ny, S.pad.nz, S.R});
    if (it != c->tuned.end()) k.add(it->second.first).add(it->second.second);
    k.add(c->xchunk3).add(c->rpl3).add(c->remap3).add(c->deep3).add(c->vz3);
}

// Enqueue a schedule: directly, or (graphs on) by replaying the graph
// captured for `key`, capturing it first if needed.  `issue(tables)` enqueues
// every launch of the schedule; batched runs get a device table buffer owned
// by the graph (filled once after the capture) in place of per-launch copies.
template <class Issue>
void run_schedule(fwi_ctx *c, hipStream_t caller, const std::string &key, size_t table_bytes, Issue &&issue)
{
    if (!c->graphs) {
        issue((char *)nullptr, caller);
        return;
    }
    hipStream_t st = caller;
    if (!caller) {
        if (!c->gstream) {
            HIPCHK(hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking));
            HIPCHK(hipEventCreateWithFlags(&c->gfence[0], hipEventDisableTiming));
            HIPCHK(hipEventCreateWithFlags(&c->gfence[1], hipEventDisableTiming));
        }
        st = c->gstream;
        HIPCHK(hipEventRecord(c->gfence[0], caller));
        HIPCHK(hipStreamWaitEvent(st, c->gfence[0], 0));
    }
    auto it = c->gcache.find(key);
    if (it != c->gcache.end() && it->second.gen != g_alloc_gen) {
        if (it->second.exec) (void)hipGraphExecDestroy(it->second.exec);
        if (it->second.tables) (void)hipFree(it->second.tables);
        c->gcache.erase(it);
        it = c->gcache.end();
    }
    if (it == c->gcache.end()) {
        fwi_ctx::GraphEntry ge;
        if (table_bytes && hipMalloc((void **)&ge.tables, table_bytes) != hipSuccess) {
            (void)hipGetLastError();
            throw Error{FWI_ENOMEM, "allocation of captured launch tables failed"};
        }
        const fwi_stats before = c->stats;
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        c->capturing = true;
        try {
            issue(ge.tables, st);
        } catch (...) {
            c->capturing = false;
            (void)hipStreamEndCapture(st, &g);
            if (g) (void)hipGraphDestroy(g);
            if (ge.tables) (void)hipFree(ge.tables);
            throw;
        }
        c->capturing = false;
        HIPCHK(hipStreamEndCapture(st, &g));
        const hipError_t e = hipGraphInstantiate(&ge.exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            if (ge.tables) (void)hipFree(ge.tables);
            throw Error{FWI_EHIP, std::string("graph instantiation failed: ") + hipGetErrorString(e)};
        }
        if (table_bytes)
            HIPCHK(hipMemcpy(ge.tables, c->btab.host, c->btab.used, hipMemcpyHostToDevice));
        ge.gen = g_alloc_gen;
        ge.n_forward = c->stats.n_forward - before.n_forward;
        ge.n_adjoint = c->stats.n_adjoint - before.n_adjoint;
        ge.n_encode = c->stats.n_encode - before.n_encode;
        ge.n_decode = c->stats.n_decode - before.n_decode;
        ge.ckpt_raw_bytes = c->stats.ckpt_raw_bytes - before.ckpt_raw_bytes;
        ge.ckpt_bytes_host = c->stats.ckpt_bytes - before.ckpt_bytes;
        it = c->gcache.emplace(key, ge).first;
        c->stats.graphs_captured += 1;
    } else {
        c->stats.graphs_replayed += 1;
        const fwi_ctx::GraphEntry &ge = it->second;
        c->stats.n_forward += ge.n_forward;
        c->stats.n_adjoint += ge.n_adjoint;
        c->stats.n_encode += ge.n_encode;
        c->stats.n_decode += ge.n_decode;
        c->stats.ckpt_raw_bytes += ge.ckpt_raw_bytes;
        c->stats.ckpt_bytes += ge.ckpt_bytes_host;
    }
    HIPCHK(hipGraphLaunch(it->second.exec, st));
    if (!caller) {
        HIPCHK(hipEventRecord(c->gfence[1], st));
        HIPCHK(hipStreamWaitEvent(caller, c->gfence[1], 0));
    }
}

}  // namespace

namespace {

// Times `steps` forward (adj = false) or adjoint launches of one launch
// shape on the context's working fields, alternating the buffer roles the
// way the sweeps rotate them, after one untimed launch.  The fields must
// hold data (see fill_tuning_fields).
double time_shape(fwi_ctx *c, Exec &ex, const fwi_shot *shot, const fwi_ctx::Shape &sh, bool adj, int steps,
                  hipEvent_t e0, hipEvent_t e1, hipStream_t st)
{
    StepParams p = ex.params();
    p.xchunk = sh.xchunk;
    p.rpl = sh.rpl;
    p.remap = sh.remap;
    p.deep = sh.deep;
    p.vz = sh.vz;
    p.rpl = shape_rpl(p.vz, p.rpl, ex.S.R);
    auto one = [&](int i) {
        float *a = (i & 1) ? c->sb.fb.p : c->sb.fa.p, *b = (i & 1) ? c->sb.fa.p : c->sb.fb.p;
        if (adj) {
            float *l1 = (i & 1) ? c->sb.lb.p : c->sb.la.p, *l2 = (i & 1) ? c->sb.la.p : c->sb.lb.p;
            p.u1 = l1; p.u2 = l2; p.out = l2; p.uk = a; p.g = c->sb.gacc.p;
        } else {
            p.u1 = a; p.u2 = b; p.out = b; p.wav = shot->wavelet; p.step = 0;
        }
        launch_step(p, ex.S.ndim, ex.S.R, adj, st);
    };
    one(0);
    HIPCHK(hipEventRecord(e0, st));
    for (int i = 0; i < steps; ++i) one(i + 1);
    HIPCHK(hipEventRecord(e1, st));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    return (double)ms / steps;
}

// The timed fields hold data (copies of the coefficient field), not zeros:
// all-zero traffic ran measurably faster and ranked the shapes differently
// from a real sweep.
void fill_tuning_fields(fwi_ctx *c, Exec &ex, hipStream_t st)
{
    HIPCHK(hipMemsetAsync(c->sb.arena.p, 0, c->sb.arena.n, st));
    ex.init_fields();
    const size_t ne = c->sb.padded_elems;
    for (float *f : {c->sb.fa.p, c->sb.fb.p, c->sb.la.p, c->sb.lb.p, c->sb.gacc.p})
        launch_copy(f, c->sb.coef.p, ne, st);
}

bool valid_shape(int ndim, const fwi_ctx::Shape &s)
{
    if (s.xchunk < 1) return false;
    if (ndim == 2) return true;
    return (s.rpl == 2 || s.rpl == 4) && s.remap >= 0 && s.remap <= 4 && (s.vz == 1 || s.vz == 2) &&
           (s.deep == 0 || (s.deep == 1 && s.vz == 1));
}


}  // namespace

namespace {

// Stacking of batched shot gradients into one array (fwi_stack): one
// StackMap per shot, validated against the target dims.
std::vector<StackMap> stack_maps(const fwi_stack *sk, const std::vector<Setup> &setups)
{
    if (!sk || !sk->origin) throw Error{FWI_EINVAL, "stack description or origins are null"};
    const int nd = setups[0].ndim;
    if (sk->ndim != nd) throw Error{FWI_EINVAL, "stack ndim differs from the shots'"};
    if (sk->region != 0 && sk->region != 1) throw Error{FWI_EINVAL, "stack region must be 0 or 1"};
    for (int d = 0; d < nd; ++d)
        if (sk->n[d] < 1) throw Error{FWI_EINVAL, "stack dims must be >= 1"};
    std::vector<StackMap> out;
    for (size_t i = 0; i < setups.size(); ++i) {
        const Setup &S = setups[i];
        StackMap m{};
        m.pm.nx = S.pad.nx;
        m.pm.ny = S.pad.ny;
        m.pm.nz = S.pad.nz;
        m.pm.sx = S.pad.sx;
        m.pm.sy = nd == 3 ? S.pad.sy : 0;
        m.pm.origin = S.pad.origin;
        const long comp[3] = {S.pad.nx, S.pad.ny, S.pad.nz};
        const int axis[3] = {0, nd == 3 ? 1 : -1, nd == 3 ? 2 : 1};   // target/origin index per (x, y, z)
        for (int a = 0; a < 3; ++a) {
            if (axis[a] < 0) {
                m.r[a] = 0;
                m.n[a] = 1;
                m.o[a] = 0;
                continue;
            }
            const long lay = sk->region ? S.nbl : 0;
            m.r[a] = lay;
            m.n[a] = comp[a] - 2 * lay;
            m.o[a] = sk->origin[i * (size_t)nd + axis[a]];
            if (m.o[a] < 0 || m.o[a] + m.n[a] > sk->n[axis[a]])
                throw Error{FWI_EINVAL, "shot " + std::to_string(i) + " falls outside the stacked gradient"};
        }
        if (nd == 3) {
            m.d0 = (long)sk->n[1] * sk->n[2];
            m.d1 = sk->n[2];
        } else {
            m.d0 = sk->n[1];
            m.d1 = 0;
        }
        out.push_back(m);
    }
    return out;
}

// per-shot gradients unpadded into grads[i], or (stacking) the target
// cleared and every shot's region added in shot order
void finish_gradients(fwi_ctx *c, std::vector<Exec> &ex, float *const *grads, const std::vector<StackMap> &smaps,
                      const fwi_stack *sk, float *gstack, hipStream_t st)
{
    const size_t n = ex.size();
    if (!sk) {
        for (size_t i = 0; i < n; ++i) launch_unpad(c->batch[i]->gacc.p, grads[i], ex[i].padmap(), st);
        return;
    }
    size_t tot = 1;
    for (int d = 0; d < sk->ndim; ++d) tot *= (size_t)sk->n[d];
    launch_fill_zero(gstack, tot, st);
    for (size_t i = 0; i < n; ++i) launch_stack_add(c->batch[i]->gacc.p, gstack, smaps[i], st);
}

}  // namespace

void fwi::set_last_error(const char *msg) { g_err = msg; }

// ================================================================== C ABI
extern "C" {

const char *fwi_last_error(void) { return g_err.c_str(); }

int fwi_ctx_create(fwi_ctx **ctx, int device, size_t pool_bytes)
{
    return guarded([&] {
        if (!ctx) throw Error{FWI_EINVAL, "ctx is null"};
        int n = 0;
        HIPCHK(hipGetDeviceCount(&n));
        if (device < 0 || device >= n) throw Error{FWI_EINVAL, "no such device"};
        HIPCHK(hipSetDevice(device));
        int resident[2][2];
        for (int d3 = 0; d3 < 2; ++d3)
            for (int enc = 0; enc < 2; ++enc) resident[d3][enc] = codec_resident_waves(d3 ? 3 : 2, enc != 0);
        fwi_ctx *c = new fwi_ctx();
        std::memcpy(c->resident, resident, sizeof resident);
        c->device = device;
        c->pool_default = pool_bytes;
        {
            std::lock_guard<std::mutex> lock(g_ctx_mu);
            g_live_ctx.insert(c);
        }
        if (const char *e = std::getenv("FWI_XCHUNK")) c->xchunk3 = std::atoi(e);
        if (const char *e = std::getenv("FWI_RPL")) c->rpl3 = std::atoi(e) == 4 ? 4 : 2;
        if (const char *e = std::getenv("FWI_REMAP")) c->remap3 = std::max(0, std::min(std::atoi(e), 4));
        if (const char *e = std::getenv("FWI_DEEP")) c->deep3 = std::atoi(e) != 0;
        if (const char *e = std::getenv("FWI_VZ")) c->vz3 = std::atoi(e) == 2 ? 2 : 1;
        if (const char *e = std::getenv("FWI_CODEC_WAVES")) c->codec_waves = std::atoi(e);
        *ctx = c;
    });
}

int fwi_ctx_destroy(fwi_ctx *c)
{
    return guarded([&] {
        if (!c) return;
        {
            std::lock_guard<std::mutex> lock(g_ctx_mu);
            g_live_ctx.erase(c);
        }
        (void)hipSetDevice(c->device);
        (void)hipDeviceSynchronize();
        for (auto &ts : c->tape_cache) ts.release();
        c->tape_cache.clear();
        for (auto e : c->evpool) (void)hipEventDestroy(e);
        for (auto e : c->spool) (void)hipEventDestroy(e);
        if (c->cstream) (void)hipStreamDestroy(c->cstream);
        if (c->t0) (void)hipEventDestroy(c->t0);
        if (c->t1) (void)hipEventDestroy(c->t1);
        c->drop_graphs();
        if (c->gstream) (void)hipStreamDestroy(c->gstream);
        for (auto e : c->gfence)
            if (e) (void)hipEventDestroy(e);
        c->pool.release(); c->sb.release();
        for (auto &b : c->batch) b->release();
        c->batch.clear();
        c->btab.release();
        c->scratch.release(); c->chunk_bits.release(); c->chunk_off.release();
        c->misc.release(); c->flags.release();
        delete c;
    });
}

int fwi_ctx_set_overlap(fwi_ctx *c, int on)
{
    return guarded([&] {
        if (!c) throw Error{FWI_EINVAL, "ctx is null"};
        c->overlap = on != 0;
        c->drop_graphs();
    });
}

int fwi_ctx_set_graphs(fwi_ctx *c, int on)
{
    return guarded([&] {
        if (!c) throw Error{FWI_EINVAL, "ctx is null"};
        HIPCHK(hipSetDevice(c->device));
        c->graphs = on != 0;
        if (!c->graphs) c->drop_graphs();
    });
}

int fwi_ctx_set_timing(fwi_ctx *c, int on)
{
    return guarded([&] {
        if (!c) throw Error{FWI_EINVAL, "ctx is null"};
        c->timing = on != 0;
    });
}

int fwi_ctx_stats(const fwi_ctx *c, fwi_stats *out)
{
    return guarded([&] {
        if (!c || !out) throw Error{FWI_EINVAL, "null argument"};
        *out = c->stats;
    });
}

int fwi_forward(fwi_ctx *c, const fwi_grid *g, const float *m, const fwi_shot *shot, float *d_sim,
                hipStream_t st)
{
    return guarded([&] {
        if (!c || !m || (!d_sim && shot && shot->nrec > 0)) throw Error{FWI_EINVAL, "null argument"};
        begin_call(c, st);
        Exec ex{c, make_setup(g, shot, true), st, m, shot};
        ensure_fields(&c->sb, ex.S);
        ex.dsim = d_sim;
        ex.init_fields();
        ex.advance(0, ex.S.nt, true);
        ex.flush_record();
        HIPCHK(hipGetLastError());
        end_call(c, st);
    });
}

int fwi_forward_state(fwi_ctx *c, const fwi_grid *g, const float *m, const fwi_shot *shot,
                      float *d_sim, float *u_last, float *u_prev, hipStream_t st)
{
    return guarded([&] {
        if (!c || !m || (!d_sim && shot && shot->nrec > 0)) throw Error{FWI_EINVAL, "null argument"};
        begin_call(c, st);
        Exec ex{c, make_setup(g, shot, true), st, m, shot};
        ensure_fields(&c->sb, ex.S);
        ex.dsim = d_sim;
        ex.init_fields();
        ex.advance(0, ex.S.nt, true);
        ex.flush_record();
        if (u_last) launch_unpad(ex.cur, u_last, ex.padmap(), st);
        if (u_prev) launch_unpad(ex.prev, u_prev, ex.padmap(), st);
        HIPCHK(hipGetLastError());
        end_call(c, st);
    });
}

int fwi_gradient(fwi_ctx *c, const fwi_grid *g, const float *m, const fwi_shot *shot,
                 const float *d_obs, const fwi_ckpt_cfg *cfg, float *grad, double *phi,
                 hipStream_t st)
{
    return guarded([&] {
        if (!c || !m || !grad || !phi || (!d_obs && shot && shot->nrec > 0))
            throw Error{FWI_EINVAL, "null argument"};
        check_cfg(cfg);
        begin_call(c, st);
        Exec ex{c, make_setup(g, shot, true), st, m, shot};
        ensure_fields(&c->sb, ex.S);
        const auto &acts = plan_for(c, ex.S.nt, cfg->nslots);
        const int used = max_slot_used(acts);
        FieldView fv = padded_view(ex.S);
        if (cfg->compress) ensure_codec(c, fv, 2 * used);
        if (c->pool.n < c->pool_default) c->pool.ensure(c->pool_default);
        const size_t cap = cfg->pool_bytes ? std::min(cfg->pool_bytes, c->pool_default) : c->pool_default;
        reset_status(c, st);
        setup_ckpt(ex, cfg, c->pool.p, cap, c->sb.slots.p, used);
        const size_t nd = (size_t)ex.S.nt * ex.S.nrec;
        c->sb.dsim.ensure(std::max<size_t>(nd, 1));
        c->sb.res.ensure(std::max<size_t>(nd, 1));
        c->sb.partials.ensure(256);
        c->sb.phi.ensure(1);
        HIPCHK(hipMemsetAsync(c->sb.phi.p, 0, sizeof(double), st));
        ex.dsim = c->sb.dsim.p;
        // captured schedules read the observed data from the context's copy
        // and leave the gradient in the padded accumulator (unpadded after the
        // replay): the graph does not depend on the caller's buffers
        if (c->graphs && nd) {
            c->sb.obs.ensure(nd);
            HIPCHK(hipMemcpyAsync(c->sb.obs.p, d_obs, nd * sizeof(float), hipMemcpyDeviceToDevice, st));
        }
        ex.d_obs = c->graphs && nd ? c->sb.obs.p : d_obs;
        ex.grad = grad;
        ex.init_fields();
        ex.init_adjoint();
        KeyBuilder key;
        key.add('G');
        key_shot(key, c, g, shot, ex.S);
        key.add(ex.d_obs).add(cfg->nslots).add(cfg->compress).add(cfg->atol).add(cap);
        run_schedule(c, st, key.s, 0, [&](char *, hipStream_t rs) {
            ex.st = rs;
            ex.run(acts, restart_flags(acts), 0, false);
            if (!c->graphs) launch_unpad(c->sb.gacc.p, grad, ex.padmap(), rs);
            ex.st = st;
        });
        if (c->graphs) launch_unpad(c->sb.gacc.p, grad, ex.padmap(), st);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(phi, c->sb.phi.p, sizeof(double), hipMemcpyDeviceToHost, st));
        finish_status(c, st);
        end_call(c, st);
    });
}

int fwi_gradient_subsampled(fwi_ctx *c, const fwi_grid *g, const float *m, const fwi_shot *shot,
                            const float *d_obs, int factor, int phase, size_t pool_bytes, float *grad,
                            double *phi, hipStream_t st)
{
    return guarded([&] {
        if (!c || !m || !grad || !phi || (!d_obs && shot && shot->nrec > 0))
            throw Error{FWI_EINVAL, "null argument"};
        if (factor < 1 || phase < 0 || phase >= factor)
            throw Error{FWI_EINVAL, "need factor >= 1 and 0 <= phase < factor"};
        begin_call(c, st);
        Exec ex{c, make_setup(g, shot, true), st, m, shot};
        ensure_fields(&c->sb, ex.S);
        size_t nstore = 0;
        for (int k = 1; k <= ex.S.nt; ++k) nstore += k % factor == phase;
        const size_t raw = c->sb.padded_elems * sizeof(float);
        if (c->pool.n < c->pool_default) c->pool.ensure(c->pool_default);
        const size_t cap = pool_bytes ? std::min(pool_bytes, c->pool_default) : c->pool_default;
        if (nstore * raw > cap)
            throw Error{FWI_ECAPACITY, "subsampled snapshots exceed the pool (" + std::to_string(nstore) +
                                           " fields): raise the factor or the pool"};
        const size_t nd = (size_t)ex.S.nt * ex.S.nrec;
        c->sb.dsim.ensure(std::max<size_t>(nd, 1));
        c->sb.res.ensure(std::max<size_t>(nd, 1));
        c->sb.partials.ensure(256);
        c->sb.phi.ensure(1);
        HIPCHK(hipMemsetAsync(c->sb.phi.p, 0, sizeof(double), st));
        ex.dsim = c->sb.dsim.p;
        ex.d_obs = d_obs;
        ex.grad = grad;
        ex.init_fields();
        ex.init_adjoint();
        ex.run_subsampled(factor, phase, (char *)c->pool.p, raw);
        launch_unpad(c->sb.gacc.p, grad, ex.padmap(), st);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(phi, c->sb.phi.p, sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        c->stats.ckpt_raw_bytes = (long long)(nstore * (size_t)ex.S.ncomp * 4);
        c->stats.ckpt_bytes = (long long)(nstore * raw);
        c->stats.pool_high = (long long)(nstore * raw);
        end_call(c, st);
    });
}

int fwi_forward_span(fwi_ctx *c, const fwi_grid *g, const float *m, const fwi_shot *shot, int k0, int k1,
                     float *u_cur, float *u_prev, float *d_sim, hipStream_t st)
{
    return guarded([&] {
        if (!c || !m || !u_cur || !u_prev || !g) throw Error{FWI_EINVAL, "null argument"};
        if (u_cur == u_prev || (d_sim && (d_sim == u_cur || d_sim == u_prev)))
            throw Error{FWI_EINVAL, "u_cur, u_prev and d_sim must be distinct arrays"};
        if (k0 < 0 || k1 < k0 || k1 > g->nt) throw Error{FWI_EINVAL, "need 0 <= k0 <= k1 <= nt"};
        begin_call(c, st);
        Exec ex{c, make_setup(g, shot, true), st, m, shot};
        ensure_fields(&c->sb, ex.S);
        const bool record = d_sim != nullptr;
        ex.dsim = d_sim;
        ex.init_fields();
        launch_pad(u_cur, ex.W0(), ex.padmap(), st);
        launch_pad(u_prev, ex.W1(), ex.padmap(), st);
        ex.work = k0;
        ex.reached = k0;
        if (k1 > k0) ex.advance(k0, k1, record);
        if (record) ex.flush_record();
        launch_unpad(ex.cur, u_cur, ex.padmap(), st);
        launch_unpad(ex.prev, u_prev, ex.padmap(), st);
        HIPCHK(hipGetLastError());
        end_call(c, st);
    });
}

static int gradient_batch_impl(fwi_ctx *c, int nshots, const fwi_grid *grids, const float *const *models,
                               const fwi_shot *shots, const float *const *d_obs, const fwi_ckpt_cfg *cfg,
                               float *const *grads, const fwi_stack *sk, float *gstack, double *phis,
                               hipStream_t st)
{
    return guarded([&] {
        if (!c || nshots < 1 || !grids || !models || !shots || !phis || !d_obs || (sk ? !gstack : !grads))
            throw Error{FWI_EINVAL, "null argument or nshots < 1"};
        check_cfg(cfg);
        for (int i = 0; i < nshots; ++i) {
            if (!models[i] || (!sk && !grads[i]) || (!d_obs[i] && shots[i].nrec > 0))
                throw Error{FWI_EINVAL, "null model, gradient or data of shot " + std::to_string(i)};
            const fwi_grid &a = grids[0], &b = grids[i];
            if (b.ndim != a.ndim || b.space_order != a.space_order || b.nt != a.nt || b.dt != a.dt)
                throw Error{FWI_EINVAL, "batched shots must share ndim, space order, nt and dt"};
        }
        begin_call(c, st);
        std::vector<Setup> setups;
        setups.reserve(nshots);
        for (int i = 0; i < nshots; ++i) setups.push_back(make_setup(&grids[i], &shots[i], true));
        const std::vector<StackMap> smaps = sk ? stack_maps(sk, setups) : std::vector<StackMap>();
        while ((int)c->batch.size() < nshots) c->batch.push_back(std::make_unique<ShotBufs>());
        const int nt = setups[0].nt;
        const auto &acts = plan_for(c, nt, cfg->nslots);
        const int used = max_slot_used(acts);
        const std::vector<char> both = restart_flags(acts);
        if (c->pool.n < c->pool_default) c->pool.ensure(c->pool_default);
        const size_t cap = cfg->pool_bytes ? std::min(cfg->pool_bytes, c->pool_default) : c->pool_default;
        // pool regions in proportion to each shot's padded field size
        std::vector<size_t> off(nshots + 1, 0);
        double wsum = 0;
        for (auto &S : setups) wsum += (double)S.pad.elems();
        double acc = 0;
        for (int i = 0; i < nshots; ++i) {
            acc += (double)setups[i].pad.elems();
            off[i + 1] = i + 1 == nshots ? cap : ((size_t)((double)cap * (acc / wsum)) & ~(size_t)255);
        }
        // codec scratch: one region per shot (the shots' fields are encoded
        // in one launch)
        std::vector<size_t> scr_off(nshots + 1, 0), cb_off(nshots + 1, 0), co_off(nshots + 1, 0);
        for (int i = 0; i < nshots; ++i) {
            const FieldView fv = padded_view(setups[i]);
            const CodecGeom cg = codec_geom(fv.ndim, fv.n);
            scr_off[i + 1] = scr_off[i] + (size_t)cg.nchunks * cg.max_chunk_words;
            cb_off[i + 1] = cb_off[i] + (size_t)cg.nchunks;
            co_off[i + 1] = co_off[i] + (size_t)((cg.nchunks + 1023) / 1024) + 2;
        }
        if (cfg->compress) {
            c->scratch.ensure(scr_off[nshots]);
            c->chunk_bits.ensure(cb_off[nshots]);
            c->chunk_off.ensure(co_off[nshots]);
        }
        c->misc.ensure(4);
        c->flags.ensure(1);
        reset_status(c, st);
        std::vector<Exec> ex;
        ex.reserve(nshots);
        for (int i = 0; i < nshots; ++i) {
            ShotBufs *b = c->batch[i].get();
            ensure_fields(b, setups[i]);
            b->slots.ensure((size_t)std::max(2 * used, 1));
            b->misc.ensure(4);
            HIPCHK(hipMemsetAsync(b->misc.p, 0, 4 * sizeof(unsigned long long), st));
            Exec e{c, setups[i], st, models[i], &shots[i], b};
            e.misc = b->misc.p;
            if (cfg->compress) {
                e.scr = c->scratch.p + scr_off[i];
                e.cbits = c->chunk_bits.p + cb_off[i];
                e.coff = c->chunk_off.p + co_off[i];
            }
            setup_ckpt(e, cfg, c->pool.p + off[i], off[i + 1] - off[i], b->slots.p, used);
            const size_t nd = (size_t)nt * e.S.nrec;
            b->dsim.ensure(std::max<size_t>(nd, 1));
            b->res.ensure(std::max<size_t>(nd, 1));
            b->partials.ensure(256);
            b->phi.ensure(1);
            HIPCHK(hipMemsetAsync(b->phi.p, 0, sizeof(double), st));
            e.dsim = b->dsim.p;
            // captured schedules read the shot's copy of the observed data
            // (the graph does not depend on the caller's buffers)
            if (c->graphs && nd) {
                b->obs.ensure(nd);
                HIPCHK(hipMemcpyAsync(b->obs.p, d_obs[i], nd * sizeof(float), hipMemcpyDeviceToDevice, st));
            }
            e.d_obs = c->graphs && nd ? b->obs.p : d_obs[i];
            e.grad = grads ? grads[i] : gstack;
            e.init_fields();
            e.init_adjoint();
            ex.push_back(std::move(e));
        }
        const size_t nbytes_tab = table_bytes_of(acts, (size_t)nshots);
        KeyBuilder key;
        key.add('B').add(nshots).add(cfg->nslots).add(cfg->compress).add(cfg->atol).add(cap);
        for (int i = 0; i < nshots; ++i) {
            key_shot(key, c, &grids[i], &shots[i], setups[i]);
            key.add(ex[i].d_obs);
        }
        c->btab.ensure(nbytes_tab);     // before any capture: it may allocate
        // the gradients leave the padded accumulators after the schedule
        // (captured schedules stop at the accumulators)
        run_schedule(c, st, key.s, nbytes_tab, [&](char *gtab, hipStream_t rs) {
            c->btab.used = 0;
            for (auto &e : ex) e.st = rs;
            BatchExec bx{c, rs, ex, setups[0].ndim, setups[0].R, gtab ? gtab : c->btab.dev.p, gtab == nullptr, {}};
            bx.run(acts, both);
            if (!c->graphs) finish_gradients(c, ex, grads, smaps, sk, gstack, rs);
            for (auto &e : ex) e.st = st;
        });
        if (c->graphs) finish_gradients(c, ex, grads, smaps, sk, gstack, st);
        std::vector<double> ph(nshots, 0.0);
        std::vector<unsigned long long> mc(4 * (size_t)nshots, 0);
        for (int i = 0; i < nshots; ++i) {
            ShotBufs *b = c->batch[i].get();
            HIPCHK(hipMemcpyAsync(&ph[i], b->phi.p, sizeof(double), hipMemcpyDeviceToHost, st));
            HIPCHK(hipMemcpyAsync(&mc[4 * i], b->misc.p, 4 * sizeof(unsigned long long),
                                  hipMemcpyDeviceToHost, st));
        }
        HIPCHK(hipGetLastError());
        finish_status(c, st);
        long long high = 0, bytes = 0;
        for (int i = 0; i < nshots; ++i) {
            phis[i] = ph[i];
            high += (long long)mc[4 * i + 1];
            bytes += (long long)mc[4 * i + 2];
        }
        if (cfg->compress) {
            c->stats.pool_high = high;
            c->stats.ckpt_bytes = bytes;
        }
        end_call(c, st);
    });
}

int fwi_gradient_batch(fwi_ctx *c, int nshots, const fwi_grid *grids, const float *const *models,
                       const fwi_shot *shots, const float *const *d_obs, const fwi_ckpt_cfg *cfg,
                       float *const *grads, double *phis, hipStream_t st)
{
    return gradient_batch_impl(c, nshots, grids, models, shots, d_obs, cfg, grads, nullptr, nullptr, phis, st);
}

int fwi_gradient_stack(fwi_ctx *c, int nshots, const fwi_grid *grids, const float *const *models,
                       const fwi_shot *shots, const float *const *d_obs, const fwi_ckpt_cfg *cfg,
                       const fwi_stack *stack, float *grad, double *phis, hipStream_t st)
{
    if (!stack) return guarded([] { throw Error{FWI_EINVAL, "stack description is null"}; });
    return gradient_batch_impl(c, nshots, grids, models, shots, d_obs, cfg, nullptr, stack, grad, phis, st);
}

// per-shot codec scratch regions of a batched call (offsets in words / entries)
static void batch_codec_scratch(fwi_ctx *c, const std::vector<Setup> &setups, bool compress,
                                std::vector<size_t> &scr_off, std::vector<size_t> &cb_off,
                                std::vector<size_t> &co_off)
{
    const size_t n = setups.size();
    scr_off.assign(n + 1, 0);
    cb_off.assign(n + 1, 0);
    co_off.assign(n + 1, 0);
    for (size_t i = 0; i < n; ++i) {
        const FieldView fv = padded_view(setups[i]);
        const CodecGeom cg = codec_geom(fv.ndim, fv.n);
        scr_off[i + 1] = scr_off[i] + (size_t)cg.nchunks * cg.max_chunk_words;
        cb_off[i + 1] = cb_off[i] + (size_t)cg.nchunks;
        co_off[i + 1] = co_off[i] + (size_t)((cg.nchunks + 1023) / 1024) + 2;
    }
    if (compress) {
        c->scratch.ensure(scr_off[n]);
        c->chunk_bits.ensure(cb_off[n]);
        c->chunk_off.ensure(co_off[n]);
    }
    c->misc.ensure(4);
    c->flags.ensure(1);
}

static void check_batch_shots(int nshots, const fwi_grid *grids)
{
    for (int i = 1; i < nshots; ++i) {
        const fwi_grid &a = grids[0], &b = grids[i];
        if (b.ndim != a.ndim || b.space_order != a.space_order || b.nt != a.nt || b.dt != a.dt)
            throw Error{FWI_EINVAL, "batched shots must share ndim, space order, nt and dt"};
    }
}

// pool high-water mark (sum over the shots) and checkpoint bytes stored
// so far on a batched tape: each shot's counters live in its own buffer
static void tape_pool_totals(const fwi_tape *t, hipStream_t st, long long *high, long long *bytes)
{
    std::vector<unsigned long long> mc(4 * t->shots.size(), 0);
    for (size_t i = 0; i < t->shots.size(); ++i)
        HIPCHK(hipMemcpyAsync(&mc[4 * i], t->shots[i]->misc.p, 4 * sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    *high = *bytes = 0;
    for (size_t i = 0; i < t->shots.size(); ++i) {
        *high += (long long)mc[4 * i + 1];
        *bytes += (long long)mc[4 * i + 2];
    }
}

int fwi_forward_ckpt_batch(fwi_ctx *c, int nshots, const fwi_grid *grids, const float *const *models,
                           const fwi_shot *shots, const fwi_ckpt_cfg *cfg, float *const *d_sim,
                           fwi_tape **tape, hipStream_t st)
{
    return guarded([&] {
        if (!c || nshots < 1 || !grids || !models || !shots || !d_sim || !tape)
            throw Error{FWI_EINVAL, "null argument or nshots < 1"};
        check_cfg(cfg);
        for (int i = 0; i < nshots; ++i)
            if (!models[i] || (!d_sim[i] && shots[i].nrec > 0))
                throw Error{FWI_EINVAL, "null model or data of shot " + std::to_string(i)};
        check_batch_shots(nshots, grids);
        begin_call(c, st);
        std::vector<Setup> setups;
        for (int i = 0; i < nshots; ++i) setups.push_back(make_setup(&grids[i], &shots[i], true));
        while ((int)c->batch.size() < nshots) c->batch.push_back(std::make_unique<ShotBufs>());
        std::unique_ptr<fwi_tape> t(new fwi_tape());
        try {
            t->ctx = c;
            t->cfg = *cfg;
            t->acts = plan_for(c, setups[0].nt, cfg->nslots);
            t->both = restart_flags(t->acts);
            const int used = max_slot_used(t->acts);
            // each shot's pool: the total split in proportion to field sizes
            const size_t cap = cfg->pool_bytes ? cfg->pool_bytes : c->pool_default;
            double wsum = 0;
            for (auto &S : setups) wsum += (double)S.pad.elems();
            const size_t nsl = (size_t)std::max(2 * used, 1);
            std::vector<size_t> sig;
            for (int i = 0; i < nshots; ++i) {
                ensure_fields(c->batch[i].get(), setups[i]);
                auto sh = std::make_unique<fwi_tape::Shot>();
                sh->grid = grids[i];
                sh->shot = shots[i];
                sh->rec.assign(shots[i].rec, shots[i].rec + (size_t)shots[i].nrec * grids[i].ndim);
                sh->shot.rec = sh->rec.data();
                sh->m = models[i];
                sh->cap = ((size_t)((double)cap * ((double)setups[i].pad.elems() / wsum))) & ~(size_t)255;
                const size_t pe = c->batch[i]->padded_elems;
                for (size_t b : {sh->cap + 8, nsl * sizeof(StreamSlot), 4 * sizeof(unsigned long long), pe * 4,
                                 pe * 4})
                    sig.push_back(b);
                t->shots.push_back(std::move(sh));
            }
            {
                KeyBuilder tag;
                for (int i = 0; i < nshots; ++i) key_shot(tag, c, &grids[i], &shots[i], setups[i]);
                t->tag = tag.s;
                // the buffers of an earlier batched tape of the same sizes, if any
                TapeStore rs = c->take_store(sig, t->tag);
                for (int i = 0; i < nshots && !rs.bufs.empty(); ++i) {
                    fwi_tape::Shot &sh = *t->shots[i];
                    store_take(rs, 5 * i + 0, sh.pool);
                    store_take(rs, 5 * i + 1, sh.slots);
                    store_take(rs, 5 * i + 2, sh.misc);
                    store_take(rs, 5 * i + 3, sh.xcur);
                    store_take(rs, 5 * i + 4, sh.xprev);
                }
            }
            for (int i = 0; i < nshots; ++i) {
                fwi_tape::Shot &sh = *t->shots[i];
                const size_t pe = c->batch[i]->padded_elems;
                sh.pool.ensure(sh.cap + 8);
                sh.slots.ensure(nsl);
                sh.misc.ensure(4);
                sh.xcur.ensure(pe);
                sh.xprev.ensure(pe);
            }
            std::vector<size_t> so, cb, co;
            batch_codec_scratch(c, setups, cfg->compress != 0, so, cb, co);
            reset_status(c, st);
            std::vector<Exec> ex;
            ex.reserve(nshots);
            for (int i = 0; i < nshots; ++i) {
                fwi_tape::Shot &sh = *t->shots[i];
                ShotBufs *b = c->batch[i].get();
                HIPCHK(hipMemsetAsync(sh.misc.p, 0, 4 * sizeof(unsigned long long), st));
                Exec e{c, setups[i], st, models[i], &sh.shot, b};
                e.misc = sh.misc.p;
                if (cfg->compress) {
                    e.scr = c->scratch.p + so[i];
                    e.cbits = c->chunk_bits.p + cb[i];
                    e.coff = c->chunk_off.p + co[i];
                }
                setup_ckpt(e, cfg, sh.pool.p, sh.cap, sh.slots.p, used);
                // captured schedules record into the shot's trace buffer and
                // copy out after the replay (the graph does not depend on d_sim)
                const size_t nd = (size_t)shots[i].nrec * (size_t)setups[i].nt;
                if (c->graphs && nd) {
                    b->dsim.ensure(nd);
                    b->res.ensure(nd);      // the backward's, so that it does not allocate
                }
                e.dsim = c->graphs && nd ? b->dsim.p : d_sim[i];
                e.init_fields();
                ex.push_back(std::move(e));
            }
            std::vector<char> sb;
            t->next = first_sweep(t->acts, t->both, sb);
            for (auto &sh : t->shots) sh->slot_both = sb;
            const size_t nbytes_tab = table_bytes_of(t->acts, (size_t)nshots);
            c->btab.ensure(nbytes_tab);     // before any capture: it may allocate
            KeyBuilder key;
            key.add('f').add(nshots).add(cfg->nslots).add(cfg->compress).add(cfg->atol).add(cap);
            for (int i = 0; i < nshots; ++i) {
                const fwi_tape::Shot &sh = *t->shots[i];
                key_shot(key, c, &grids[i], &shots[i], setups[i]);
                key.add(ex[i].dsim).add(sh.pool.p).add(sh.slots.p).add(sh.misc.p).add(sh.xcur.p).add(sh.xprev.p);
            }
            run_schedule(c, st, key.s, nbytes_tab, [&](char *gtab, hipStream_t rs) {
                c->btab.used = 0;
                for (auto &e : ex) e.st = rs;
                BatchExec bx{c, rs, ex, setups[0].ndim, setups[0].R, gtab ? gtab : c->btab.dev.p, gtab == nullptr, {}};
                bx.run(t->acts, t->both, 0, true);
                for (int i = 0; i < nshots; ++i) {
                    fwi_tape::Shot &sh = *t->shots[i];
                    const size_t pe = c->batch[i]->padded_elems;
                    launch_copy(sh.xcur.p, ex[i].cur, pe, rs);
                    launch_copy(sh.xprev.p, ex[i].prev, pe, rs);
                }
                for (auto &e : ex) e.st = st;
            });
            for (int i = 0; i < nshots; ++i)
                if (ex[i].dsim != d_sim[i])
                    HIPCHK(hipMemcpyAsync(d_sim[i], ex[i].dsim,
                                          (size_t)shots[i].nrec * (size_t)setups[i].nt * sizeof(float),
                                          hipMemcpyDeviceToDevice, st));
            HIPCHK(hipGetLastError());
            finish_status(c, st);
            if (cfg->compress) {
                tape_pool_totals(t.get(), st, &c->stats.pool_high, &c->stats.ckpt_bytes);
                t->fwd_bytes = c->stats.ckpt_bytes;
            }
            end_call(c, st);
        } catch (...) {
            for (auto &sh : t->shots) sh->release();
            throw;
        }
        *tape = t.release();
    });
}

static int backward_batch_impl(fwi_ctx *c, fwi_tape *t, const float *const *dd, float *const *grads,
                               const fwi_stack *sk, float *gstack, hipStream_t st)
{
    return guarded([&] {
        if (!c || !t || !dd || (sk ? !gstack : !grads)) throw Error{FWI_EINVAL, "null argument"};
        if (t->shots.empty()) throw Error{FWI_EINVAL, "a single-shot tape needs fwi_backward"};
        if (t->used) throw Error{FWI_EINVAL, "tape already back-propagated"};
        const int nshots = (int)t->shots.size();
        for (int i = 0; i < nshots; ++i)
            if ((!sk && !grads[i]) || (!dd[i] && t->shots[i]->shot.nrec > 0))
                throw Error{FWI_EINVAL, "null gradient or adjoint source of shot " + std::to_string(i)};
        begin_call(c, st);
        std::vector<Setup> setups;
        for (auto &sh : t->shots) setups.push_back(make_setup(&sh->grid, &sh->shot, true));
        const std::vector<StackMap> smaps = sk ? stack_maps(sk, setups) : std::vector<StackMap>();
        while ((int)c->batch.size() < nshots) c->batch.push_back(std::make_unique<ShotBufs>());
        const int used = max_slot_used(t->acts);
        std::vector<size_t> so, cb, co;
        batch_codec_scratch(c, setups, t->cfg.compress != 0, so, cb, co);
        reset_status(c, st);
        std::vector<Exec> ex;
        ex.reserve(nshots);
        for (int i = 0; i < nshots; ++i) {
            fwi_tape::Shot &sh = *t->shots[i];
            ShotBufs *b = c->batch[i].get();
            ensure_fields(b, setups[i]);
            Exec e{c, setups[i], st, sh.m, &sh.shot, b};
            e.misc = sh.misc.p;
            if (t->cfg.compress) {
                e.scr = c->scratch.p + so[i];
                e.cbits = c->chunk_bits.p + cb[i];
                e.coff = c->chunk_off.p + co[i];
            }
            setup_ckpt(e, &t->cfg, sh.pool.p, sh.cap, sh.slots.p, used);
            e.grad = grads ? grads[i] : gstack;
            // captured schedules read the adjoint source from the shot's
            // buffer, filled before the replay (the graph does not depend on dd)
            const size_t nd = (size_t)sh.shot.nrec * (size_t)setups[i].nt;
            if (c->graphs && nd) {
                b->res.ensure(nd);
                HIPCHK(hipMemcpyAsync(b->res.p, dd[i], nd * sizeof(float), hipMemcpyDeviceToDevice, st));
            }
            e.adj_src = c->graphs && nd ? b->res.p : dd[i];
            e.init_fields();
            e.init_adjoint();
            e.cur = sh.xcur.p;
            e.prev = sh.xprev.p;
            e.work = sh.grid.nt;
            e.reached = sh.grid.nt;
            e.slot_both = sh.slot_both;
            ex.push_back(std::move(e));
        }
        const size_t nbytes_tab = table_bytes_of(t->acts, (size_t)nshots);
        c->btab.ensure(nbytes_tab);     // before any capture: it may allocate
        KeyBuilder key;
        key.add('b').add(nshots).add(t->cfg.nslots).add(t->cfg.compress).add(t->cfg.atol).add(t->next);
        for (int i = 0; i < nshots; ++i) {
            const fwi_tape::Shot &sh = *t->shots[i];
            key_shot(key, c, &sh.grid, &sh.shot, setups[i]);
            key.add(ex[i].adj_src).add(sh.pool.p).add(sh.slots.p).add(sh.misc.p).add(sh.xcur.p).add(sh.xprev.p)
                .add(sh.cap);
        }
        // the gradients leave the padded accumulators after the schedule;
        // captured schedules stop at the accumulators, so the graph does not
        // depend on where the caller wants the gradients
        key.add(sk ? 'S' : '-');
        run_schedule(c, st, key.s, nbytes_tab, [&](char *gtab, hipStream_t rs) {
            c->btab.used = 0;
            for (auto &e : ex) e.st = rs;
            BatchExec bx{c, rs, ex, setups[0].ndim, setups[0].R, gtab ? gtab : c->btab.dev.p, gtab == nullptr, {}};
            bx.run(t->acts, t->both, t->next, false);
            if (!c->graphs) finish_gradients(c, ex, grads, smaps, sk, gstack, rs);
            for (auto &e : ex) e.st = st;
        });
        if (c->graphs) finish_gradients(c, ex, grads, smaps, sk, gstack, st);
        HIPCHK(hipGetLastError());
        finish_status(c, st);
        if (t->cfg.compress) {
            long long total = 0;
            tape_pool_totals(t, st, &c->stats.pool_high, &total);
            c->stats.ckpt_bytes = total - t->fwd_bytes;
        }
        t->used = true;
        end_call(c, st);
    });
}

int fwi_backward_batch(fwi_ctx *c, fwi_tape *t, const float *const *dd, float *const *grads, hipStream_t st)
{
    return backward_batch_impl(c, t, dd, grads, nullptr, nullptr, st);
}

int fwi_backward_stack(fwi_ctx *c, fwi_tape *t, const float *const *dd, const fwi_stack *stack, float *grad,
                       hipStream_t st)
{
    if (!stack) return guarded([] { throw Error{FWI_EINVAL, "stack description is null"}; });
    return backward_batch_impl(c, t, dd, nullptr, stack, grad, st);
}

int fwi_forward_ckpt(fwi_ctx *c, const fwi_grid *g, const float *m, const fwi_shot *shot,
                     const fwi_ckpt_cfg *cfg, float *d_sim, fwi_tape **tape, hipStream_t st)
{
    return guarded([&] {
        if (!c || !m || !tape || (!d_sim && shot && shot->nrec > 0)) throw Error{FWI_EINVAL, "null argument"};
        check_cfg(cfg);
        begin_call(c, st);
        fwi_tape *t = new fwi_tape();
        try {
            t->ctx = c;
            t->grid = *g;
            t->shot = *shot;
            t->m = m;
            t->cfg = *cfg;
            Exec ex{c, make_setup(g, shot, true), st, m, shot};
            t->rec.assign(shot->rec, shot->rec + (size_t)shot->nrec * g->ndim);
            t->shot.rec = t->rec.data();
            ensure_fields(&c->sb, ex.S);
            t->acts = plan_for(c, ex.S.nt, cfg->nslots);
            const int used = max_slot_used(t->acts);
            FieldView fv = padded_view(ex.S);
            if (cfg->compress) ensure_codec(c, fv, 1);
            const size_t cap = cfg->pool_bytes ? cfg->pool_bytes : c->pool_default;
            const size_t pe = c->sb.padded_elems;
            const size_t nsl = (size_t)std::max(2 * used, 1);
            {
                KeyBuilder tag;
                key_shot(tag, c, g, shot, ex.S);
                t->tag = tag.s;
                // the buffers of an earlier tape of the same sizes, if any
                TapeStore rs = c->take_store({cap + 8, nsl * sizeof(StreamSlot), pe * 4, pe * 4}, t->tag);
                if (!rs.bufs.empty()) {
                    store_take(rs, 0, t->pool);
                    store_take(rs, 1, t->slots);
                    store_take(rs, 2, t->xcur);
                    store_take(rs, 3, t->xprev);
                }
            }
            t->pool.ensure(cap + 8);
            t->slots.ensure(nsl);
            t->xcur.ensure(pe);
            t->xprev.ensure(pe);
            reset_status(c, st);
            setup_ckpt(ex, cfg, t->pool.p, cap, t->slots.p, used);
            // captured schedules record into the context's trace buffer and
            // copy out after the replay, so they do not depend on d_sim
            const size_t nd = (size_t)shot->nrec * (size_t)ex.S.nt;
            if (c->graphs && nd) {
                c->sb.dsim.ensure(nd);
                c->sb.res.ensure(nd);       // the backward's, so that it does not allocate
            }
            ex.dsim = c->graphs && nd ? c->sb.dsim.p : d_sim;
            ex.init_fields();
            t->both = restart_flags(t->acts);
            t->next = first_sweep(t->acts, t->both, t->slot_both);
            KeyBuilder key;
            key.add('F');
            key_shot(key, c, g, shot, ex.S);
            key.add(ex.dsim).add(cfg->nslots).add(cfg->compress).add(cfg->atol).add(cap);
            key.add(t->pool.p).add(t->slots.p).add(t->xcur.p).add(t->xprev.p);
            run_schedule(c, st, key.s, 0, [&](char *, hipStream_t rs) {
                ex.st = rs;
                ex.run(t->acts, t->both, 0, true);
                launch_copy(t->xcur.p, ex.cur, pe, rs);
                launch_copy(t->xprev.p, ex.prev, pe, rs);
                ex.st = st;
            });
            if (ex.dsim != d_sim)
                HIPCHK(hipMemcpyAsync(d_sim, ex.dsim, nd * sizeof(float), hipMemcpyDeviceToDevice, st));
            HIPCHK(hipGetLastError());
            finish_status(c, st);
            end_call(c, st);
        } catch (...) {
            t->pool.release(); t->slots.release(); t->xcur.release(); t->xprev.release();
            delete t;
            throw;
        }
        *tape = t;
    });
}

int fwi_backward(fwi_ctx *c, fwi_tape *t, const float *dd, float *grad, hipStream_t st)
{
    return guarded([&] {
        if (!c || !t || !grad || (!dd && t->shot.nrec > 0)) throw Error{FWI_EINVAL, "null argument"};
        if (t->used) throw Error{FWI_EINVAL, "tape already back-propagated"};
        if (!t->shots.empty()) throw Error{FWI_EINVAL, "a batched tape needs fwi_backward_batch"};
        begin_call(c, st);
        Exec ex{c, make_setup(&t->grid, &t->shot, true), st, t->m, &t->shot};
        ensure_fields(&c->sb, ex.S);
        const int used = max_slot_used(t->acts);
        FieldView fv = padded_view(ex.S);
        if (t->cfg.compress) ensure_codec(c, fv, 1);
        const size_t cap = t->cfg.pool_bytes ? t->cfg.pool_bytes : c->pool_default;
        reset_status(c, st);
        setup_ckpt(ex, &t->cfg, t->pool.p, cap, t->slots.p, used);
        ex.grad = grad;
        // captured schedules read the adjoint source from the context's
        // buffer (filled before the replay) and leave the gradient in the
        // padded accumulator, unpadded after the replay: the graph does not
        // depend on dd or grad
        const size_t nd = (size_t)t->shot.nrec * (size_t)ex.S.nt;
        if (c->graphs && nd) {
            c->sb.res.ensure(nd);
            HIPCHK(hipMemcpyAsync(c->sb.res.p, dd, nd * sizeof(float), hipMemcpyDeviceToDevice, st));
        }
        ex.adj_src = c->graphs && nd ? c->sb.res.p : dd;
        ex.init_fields();
        ex.init_adjoint();
        ex.cur = t->xcur.p;
        ex.prev = t->xprev.p;
        ex.work = t->grid.nt;
        ex.reached = t->grid.nt;
        ex.slot_both = t->slot_both;
        KeyBuilder key;
        key.add('U');
        key_shot(key, c, &t->grid, &t->shot, ex.S);
        key.add(ex.adj_src).add(t->cfg.nslots).add(t->cfg.compress).add(t->cfg.atol).add(cap);
        key.add(t->pool.p).add(t->slots.p).add(t->xcur.p).add(t->xprev.p);
        run_schedule(c, st, key.s, 0, [&](char *, hipStream_t rs) {
            ex.st = rs;
            ex.run(t->acts, t->both, t->next, false);
            if (!c->graphs) launch_unpad(c->sb.gacc.p, grad, ex.padmap(), rs);
            ex.st = st;
        });
        if (c->graphs) launch_unpad(c->sb.gacc.p, grad, ex.padmap(), st);
        HIPCHK(hipGetLastError());
        finish_status(c, st);
        t->used = true;
        end_call(c, st);
    });
}

int fwi_tape_free(fwi_tape *t)
{
    return guarded([&] {
        if (!t) return;
        // the buffers go back to the context (for the next tape of the same
        // sizes) while it lives, else to the device
        TapeStore rs;
        rs.tag = t->tag;
        if (t->shots.empty()) {
            store_put(rs, t->pool);
            store_put(rs, t->slots);
            store_put(rs, t->xcur);
            store_put(rs, t->xprev);
        } else {
            for (auto &sh : t->shots) {
                store_put(rs, sh->pool);
                store_put(rs, sh->slots);
                store_put(rs, sh->misc);
                store_put(rs, sh->xcur);
                store_put(rs, sh->xprev);
            }
        }
        bool alive;
        {
            std::lock_guard<std::mutex> lock(g_ctx_mu);
            alive = g_live_ctx.count(t->ctx) != 0;
        }
        if (alive) t->ctx->keep_store(std::move(rs));
        else rs.release();
        delete t;
    });
}

int fwi_tape_stream(fwi_tape *t, int shot, int slot, int level, void *out, size_t cap, size_t *nbytes,
                    hipStream_t st)
{
    return guarded([&] {
        if (!t || !nbytes) throw Error{FWI_EINVAL, "null argument"};
        if (!t->cfg.compress) throw Error{FWI_EINVAL, "the tape holds exact checkpoints, not streams"};
        if (level != 0 && level != 1) throw Error{FWI_EINVAL, "level must be 0 (u^k) or 1 (u^(k-1))"};
        const bool batched = !t->shots.empty();
        if (shot < 0 || shot >= (batched ? (int)t->shots.size() : 1)) throw Error{FWI_EINVAL, "no such shot"};
        const std::vector<char> &both = batched ? t->shots[shot]->slot_both : t->slot_both;
        const StreamSlot *slots = batched ? t->shots[shot]->slots.p : t->slots.p;
        const unsigned char *pool = batched ? t->shots[shot]->pool.p : t->pool.p;
        if (slot < 0 || slot >= (int)both.size()) throw Error{FWI_EINVAL, "no checkpoint in that slot"};
        if (level == 1 && !both[slot]) throw Error{FWI_EINVAL, "that checkpoint holds u^k alone"};
        HIPCHK(hipSetDevice(t->ctx->device));
        StreamSlot sl{};
        HIPCHK(hipMemcpyAsync(&sl, slots + 2 * slot + level, sizeof(sl), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (!sl.valid) throw Error{FWI_EINVAL, "no stream stored in that slot"};
        *nbytes = (size_t)sl.bytes;
        if (!out) return;
        if (cap < sl.bytes) throw Error{FWI_ECAPACITY, "output buffer smaller than the stream"};
        HIPCHK(hipMemcpyAsync(out, pool + sl.offset, (size_t)sl.bytes, hipMemcpyDeviceToDevice, st));
    });
}

int ckpt_bound(int ndim, const int n[3], size_t *max_bytes)
{
    return guarded([&] {
        if ((ndim != 2 && ndim != 3) || !n || !max_bytes) throw Error{FWI_EINVAL, "bad arguments"};
        long dims[3];
        for (int d = 0; d < ndim; ++d)
            if (n[d] < 1) throw Error{FWI_EINVAL, "dims must be >= 1"};
        dims[0] = n[0];
        dims[1] = ndim == 3 ? n[1] : 1;
        dims[2] = ndim == 3 ? n[2] : n[1];
        *max_bytes = (size_t)codec_bound(codec_geom(ndim, dims));
    });
}

int fwi_ckpt_pool_bytes(const fwi_grid *g, const fwi_ckpt_cfg *cfg, size_t *bytes)
{
    return guarded([&] {
        if (!g || !bytes) throw Error{FWI_EINVAL, "null argument"};
        check_cfg(cfg);
        if (g->ndim != 2 && g->ndim != 3) throw Error{FWI_EINVAL, "ndim must be 2 or 3"};
        if (g->nt < 1 || g->nbl < 0) throw Error{FWI_EINVAL, "nt must be >= 1 and nbl >= 0"};
        int comp[3] = {1, 1, 1};
        for (int d = 0; d < g->ndim; ++d) {
            if (g->n[d] < 1) throw Error{FWI_EINVAL, "dims must be >= 1"};
            comp[d] = g->n[d] + 2 * g->nbl;
        }
        const int used = max_slot_used(revolve_plan(g->nt, cfg->nslots));
        size_t per;
        if (cfg->compress) {
            const long dims[3] = {comp[0], g->ndim == 3 ? comp[1] : 1, g->ndim == 3 ? comp[2] : comp[1]};
            per = (size_t)codec_bound(codec_geom(g->ndim, dims)) + 512;    // placement alignment
        } else {
            per = make_padded(g->ndim, comp).elems() * sizeof(float);
        }
        *bytes = (size_t)2 * (size_t)used * per;
    });
}

static FieldView dense_view(int ndim, const int n[3])
{
    FieldView f;
    f.ndim = ndim;
    f.n[0] = n[0];
    f.n[1] = ndim == 3 ? n[1] : 1;
    f.n[2] = ndim == 3 ? n[2] : n[1];
    f.sx = f.n[1] * f.n[2];
    f.sy = ndim == 3 ? f.n[2] : 0;
    f.padded = 0;
    return f;
}

// a field inside a larger array: element (x, y, z) at origin + x sx + y sy + z
static FieldView checked_view(int ndim, const int n[3], long sx, long sy, int padded, const float *origin)
{
    if (ndim != 2 && ndim != 3) throw Error{FWI_EINVAL, "ndim must be 2 or 3"};
    for (int d = 0; d < ndim; ++d)
        if (n[d] < 1) throw Error{FWI_EINVAL, "dims must be >= 1"};
    FieldView f;
    f.ndim = ndim;
    f.n[0] = n[0];
    f.n[1] = ndim == 3 ? n[1] : 1;
    f.n[2] = ndim == 3 ? n[2] : n[1];
    f.sx = sx;
    f.sy = ndim == 3 ? sy : 0;
    f.padded = padded != 0;
    const long slack = padded ? 3 : 0;
    if (ndim == 3 ? (sy < f.n[2] + slack || sx < (f.n[1] + slack) * sy) : (sx < f.n[2] + slack))
        throw Error{FWI_EINVAL, "strides overlap rows (or leave no room for the padding declared)"};
    if (padded && ((uintptr_t)origin % 16 != 0 || sx % 4 != 0 || (ndim == 3 && sy % 4 != 0)))
        throw Error{FWI_EINVAL, "a padded view needs 16-byte aligned rows"};
    return f;
}

static void compress_view(fwi_ctx *c, const FieldView &f, const float *field, double atol, void *out,
                          size_t cap, size_t *nbytes, hipStream_t st)
{
    if (!(atol >= 2.2250738585072014e-308) || !std::isfinite(atol))
        throw Error{FWI_EINVAL, "atol must be a positive normal number"};
    begin_call(c, st);
    ensure_codec(c, f, 1);
    reset_status(c, st);
    EncodeArgs e{};
    e.f = f;
    e.src = field;
    e.atol = atol;
    e.scratch = c->scratch.p;
    e.chunk_bits = c->chunk_bits.p;
    e.chunk_off = c->chunk_off.p;
    e.dst = (unsigned char *)out;
    e.cap = cap;
    e.out_bytes = c->misc.p + 0;
    e.pool_high = c->misc.p + 1;
    e.total_bytes = c->misc.p + 2;
    e.flags = c->flags.p;
    {
        Timer tm(c, st, K_ENC);
        codec_encode(e, st);
    }
    HIPCHK(hipGetLastError());
    unsigned long long nb = 0;
    HIPCHK(hipMemcpyAsync(&nb, c->misc.p, sizeof(nb), hipMemcpyDeviceToHost, st));
    finish_status(c, st);
    *nbytes = (size_t)nb;
    c->stats.n_encode = 1;
    end_call(c, st);
}

// the 64-byte header of a stream for field f (host copy), checked against
// the field's geometry and the stream's byte count (format: Sec. 1.4 codec)
static void check_stream_header(const unsigned char *h, const FieldView &f, size_t nbytes)
{
    const int ndim = f.ndim;
    const CodecGeom g = codec_geom(ndim, f.n);
    auto u32 = [&](int o) { unsigned v; memcpy(&v, h + o, 4); return v; };
    auto u64 = [&](int o) { unsigned long long v; memcpy(&v, h + o, 8); return v; };
    const unsigned want[3] = {(unsigned)f.n[0], (unsigned)(ndim == 3 ? f.n[1] : f.n[2]),
                              (unsigned)(ndim == 3 ? f.n[2] : 1)};
    if (memcmp(h, "FWZ1", 4) != 0 || h[4] != 1 || h[5] != 0) throw Error{FWI_ECORRUPT, "bad magic or version"};
    if (h[6] != ndim || h[7] != 24 || h[20] != g.guard || h[22] != g.tp ||
        h[21] != (unsigned char)__builtin_ctz((unsigned)g.kblk))
        throw Error{FWI_ECORRUPT, "stream parameters do not match"};
    if (u32(8) != want[0] || u32(12) != want[1] || u32(16) != want[2])
        throw Error{FWI_ECORRUPT, "stream dims do not match"};
    if ((long)u32(36) != g.nchunks || (long)u64(40) != g.nblocks) throw Error{FWI_ECORRUPT, "bad tables"};
    const unsigned long long pbits = u64(48);
    const unsigned long long total = 64ull + (unsigned long long)g.table_bytes + 8ull * ((pbits + 63) / 64);
    if (u64(56) != total || nbytes < total) throw Error{FWI_ECORRUPT, "stream length mismatch"};
}

static void decompress_view(fwi_ctx *c, const FieldView &f, const void *stream, size_t nbytes, float *field,
                            hipStream_t st)
{
    begin_call(c, st);
    if (nbytes < 64) throw Error{FWI_ECORRUPT, "stream shorter than its header"};
    unsigned char h[64];
    HIPCHK(hipMemcpyAsync(h, stream, 64, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    check_stream_header(h, f, nbytes);
    reset_status(c, st);
    DecodeArgs d{};
    d.f = f;
    d.dst = field;
    d.stream = (const unsigned char *)stream;
    d.nbytes = nbytes;
    d.flags = c->flags.p;
    {
        Timer tm(c, st, K_DEC);
        codec_decode(d, st);
    }
    HIPCHK(hipGetLastError());
    finish_status(c, st);
    c->stats.n_decode = 1;
    end_call(c, st);
}

int ckpt_compress(fwi_ctx *c, const float *field, int ndim, const int n[3], double atol, void *out,
                  size_t cap, size_t *nbytes, hipStream_t st)
{
    return guarded([&] {
        if (!c || !field || !out || !nbytes || !n) throw Error{FWI_EINVAL, "null argument"};
        if (ndim != 2 && ndim != 3) throw Error{FWI_EINVAL, "ndim must be 2 or 3"};
        for (int d = 0; d < ndim; ++d)
            if (n[d] < 1) throw Error{FWI_EINVAL, "dims must be >= 1"};
        compress_view(c, dense_view(ndim, n), field, atol, out, cap, nbytes, st);
    });
}

int ckpt_compress_view(fwi_ctx *c, const float *origin, int ndim, const int n[3], long sx, long sy,
                       int padded, double atol, void *out, size_t cap, size_t *nbytes, hipStream_t st)
{
    return guarded([&] {
        if (!c || !origin || !out || !nbytes || !n) throw Error{FWI_EINVAL, "null argument"};
        compress_view(c, checked_view(ndim, n, sx, sy, padded, origin), origin, atol, out, cap, nbytes, st);
    });
}

int ckpt_decompress(fwi_ctx *c, const void *stream, size_t nbytes, float *field, int ndim, const int n[3],
                    hipStream_t st)
{
    return guarded([&] {
        if (!c || !stream || !field || !n) throw Error{FWI_EINVAL, "null argument"};
        if (ndim != 2 && ndim != 3) throw Error{FWI_EINVAL, "ndim must be 2 or 3"};
        for (int d = 0; d < ndim; ++d)
            if (n[d] < 1) throw Error{FWI_EINVAL, "dims must be >= 1"};
        decompress_view(c, dense_view(ndim, n), stream, nbytes, field, st);
    });
}

int ckpt_decompress_view(fwi_ctx *c, const void *stream, size_t nbytes, float *origin, int ndim,
                         const int n[3], long sx, long sy, int padded, hipStream_t st)
{
    return guarded([&] {
        if (!c || !stream || !origin || !n) throw Error{FWI_EINVAL, "null argument"};
        decompress_view(c, checked_view(ndim, n, sx, sy, padded, origin), stream, nbytes, origin, st);
    });
}

// dense fields of a batched codec call: field i has dims n[3 i .. 3 i + ndim)
static std::vector<FieldView> batch_views(int nfields, int ndim, const int *n)
{
    if (nfields < 1) throw Error{FWI_EINVAL, "nfields must be >= 1"};
    if (ndim != 2 && ndim != 3) throw Error{FWI_EINVAL, "ndim must be 2 or 3"};
    std::vector<FieldView> v((size_t)nfields);
    for (size_t i = 0; i < (size_t)nfields; ++i) {
        for (int d = 0; d < ndim; ++d)
            if (n[3 * i + (size_t)d] < 1) throw Error{FWI_EINVAL, "dims must be >= 1"};
        v[i] = dense_view(ndim, n + 3 * i);
    }
    return v;
}

int ckpt_compress_batch(fwi_ctx *c, int nfields, int ndim, const int *n, const float *const *fields,
                        double atol, void *const *out, const size_t *cap, size_t *nbytes, hipStream_t st)
{
    return guarded([&] {
        if (!c || !n || !fields || !out || !cap || !nbytes) throw Error{FWI_EINVAL, "null argument"};
        const std::vector<FieldView> fv = batch_views(nfields, ndim, n);
        for (int i = 0; i < nfields; ++i)
            if (!fields[i] || !out[i]) throw Error{FWI_EINVAL, "null field or output"};
        if (!(atol >= 2.2250738585072014e-308) || !std::isfinite(atol))
            throw Error{FWI_EINVAL, "atol must be a positive normal number"};
        begin_call(c, st);
        // each field's encode workspace is a slice of the context's buffers
        std::vector<size_t> o_scr(fv.size()), o_bits(fv.size()), o_tile(fv.size());
        size_t scr = 0, bits = 0, tiles = 0;
        for (size_t i = 0; i < fv.size(); ++i) {
            const CodecGeom g = codec_geom(ndim, fv[i].n);
            o_scr[i] = scr;
            o_bits[i] = bits;
            o_tile[i] = tiles;
            scr += (size_t)g.nchunks * (size_t)g.max_chunk_words;
            bits += (size_t)g.nchunks;
            tiles += (size_t)((g.nchunks + 1023) / 1024) + 2;
        }
        c->scratch.ensure(scr);
        c->chunk_bits.ensure(bits);
        c->chunk_off.ensure(tiles);
        c->misc.ensure(4 * fv.size());
        c->flags.ensure(1);
        c->btab.ensure((size_t)nfields * codec_job_bytes(true) + 256);
        HIPCHK(hipMemsetAsync(c->flags.p, 0, sizeof(unsigned int), st));
        HIPCHK(hipMemsetAsync(c->misc.p, 0, 4 * fv.size() * sizeof(unsigned long long), st));
        std::vector<EncodeArgs> args(fv.size());
        for (size_t i = 0; i < fv.size(); ++i) {
            EncodeArgs &e = args[i];
            e.f = fv[i];
            e.src = fields[i];
            e.atol = atol;
            e.scratch = c->scratch.p + o_scr[i];
            e.chunk_bits = c->chunk_bits.p + o_bits[i];
            e.chunk_off = c->chunk_off.p + o_tile[i];
            e.dst = (unsigned char *)out[i];
            e.cap = cap[i];
            e.out_bytes = c->misc.p + 4 * i;
            e.pool_high = c->misc.p + 4 * i + 1;
            e.total_bytes = c->misc.p + 4 * i + 2;
            e.flags = c->flags.p;
        }
        {
            Timer tm(c, st, K_ENC);
            const size_t off = c->btab.take((size_t)nfields * codec_job_bytes(true));
            codec_encode_batch(args.data(), nfields, c->btab.host + off, c->btab.dev.p + off, true, st);
        }
        HIPCHK(hipGetLastError());
        std::vector<unsigned long long> misc(4 * fv.size());
        unsigned int fl = 0;
        HIPCHK(hipMemcpyAsync(misc.data(), c->misc.p, misc.size() * sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(&fl, c->flags.p, sizeof(fl), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (fl & 1u) throw Error{FWI_ENONFINITE, "non-finite value in a field"};
        if (fl & 8u)
            throw Error{FWI_ERANGE, "a value at or above atol * 2^23 in a field: the fixed-accuracy bound "
                                    "cannot hold at this atol (raise atol)"};
        if (fl & 2u) throw Error{FWI_ECAPACITY, "an output buffer is smaller than its stream"};
        long long total = 0;
        for (size_t i = 0; i < fv.size(); ++i) {
            nbytes[i] = (size_t)misc[4 * i];
            total += (long long)misc[4 * i];
        }
        c->stats.ckpt_bytes = total;
        c->stats.n_encode = nfields;
        end_call(c, st);
    });
}

int ckpt_decompress_batch(fwi_ctx *c, int nfields, int ndim, const int *n, const void *const *streams,
                          const size_t *nbytes, float *const *fields, hipStream_t st)
{
    return guarded([&] {
        if (!c || !n || !streams || !nbytes || !fields) throw Error{FWI_EINVAL, "null argument"};
        const std::vector<FieldView> fv = batch_views(nfields, ndim, n);
        for (int i = 0; i < nfields; ++i) {
            if (!streams[i] || !fields[i]) throw Error{FWI_EINVAL, "null stream or field"};
            if (nbytes[i] < 64) throw Error{FWI_ECORRUPT, "stream shorter than its header"};
        }
        begin_call(c, st);
        c->flags.ensure(1);
        c->btab.ensure((size_t)nfields * codec_job_bytes(false) + 256);
        std::vector<unsigned char> h(64 * fv.size());
        for (size_t i = 0; i < fv.size(); ++i)
            HIPCHK(hipMemcpyAsync(h.data() + 64 * i, streams[i], 64, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (size_t i = 0; i < fv.size(); ++i) check_stream_header(h.data() + 64 * i, fv[i], nbytes[i]);
        HIPCHK(hipMemsetAsync(c->flags.p, 0, sizeof(unsigned int), st));
        std::vector<DecodeArgs> args(fv.size());
        for (size_t i = 0; i < fv.size(); ++i) {
            DecodeArgs &d = args[i];
            d.f = fv[i];
            d.dst = fields[i];
            d.stream = (const unsigned char *)streams[i];
            d.nbytes = nbytes[i];
            d.flags = c->flags.p;
        }
        {
            Timer tm(c, st, K_DEC);
            const size_t off = c->btab.take((size_t)nfields * codec_job_bytes(false));
            codec_decode_batch(args.data(), nfields, c->btab.host + off, c->btab.dev.p + off, true, st);
        }
        HIPCHK(hipGetLastError());
        unsigned int fl = 0;
        HIPCHK(hipMemcpyAsync(&fl, c->flags.p, sizeof(fl), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (fl & 4u) throw Error{FWI_ECORRUPT, "a stream failed to decode"};
        c->stats.n_decode = nfields;
        end_call(c, st);
    });
}

int fwi_autotune(fwi_ctx *c, const fwi_grid *g, const float *m, const fwi_shot *shot, int steps,
                 fwi_tune_result *out, hipStream_t st)
{
    return guarded([&] {
        if (!c || !m || !out) throw Error{FWI_EINVAL, "null argument"};
        if (steps < 1) throw Error{FWI_EINVAL, "steps must be >= 1"};
        HIPCHK(hipSetDevice(c->device));
        Exec ex{c, make_setup(g, shot, true), st, m, shot};
        ensure_fields(&c->sb, ex.S);
        std::vector<fwi_ctx::Shape> cands;
        const int xcs3[] = {8, 16, 32, 64};
        const int xcs2[] = {4, 8, 16, 32, 64};
        if (ex.S.ndim == 3) {
            for (int xc : xcs3) {
                for (int remap : {0, 1}) {
                    cands.push_back({xc, 2, remap, 0, 1});
                    cands.push_back({xc, 4, remap, 0, 1});
                    cands.push_back({xc, 2, remap, 1, 1});
                }
                for (int remap : {2, 3, 4}) cands.push_back({xc, 2, remap, 0, 1});
                for (int remap : {0, 1, 2}) {
                    cands.push_back({xc, 2, remap, 0, 2});
                    cands.push_back({xc, 4, remap, 0, 2});
                }
            }
            for (int remap : {0, 1, 2}) cands.push_back({128, 4, remap, 0, 2});
        } else {
            for (int xc : xcs2) cands.push_back({xc, 2, 0, 0, 1});
        }
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        auto time_it = [&](const fwi_ctx::Shape &sh, bool adj) { return time_shape(c, ex, shot, sh, adj, steps, e0, e1, st); };
        fill_tuning_fields(c, ex, st);
        // screen every candidate, then re-time the best eight of each sweep
        // three more times, interleaved
        std::vector<std::pair<double, size_t>> rf, ra;
        for (size_t i = 0; i < cands.size(); ++i) {
            rf.push_back({time_it(cands[i], false), i});
            ra.push_back({time_it(cands[i], true), i});
        }
        std::sort(rf.begin(), rf.end());
        std::sort(ra.begin(), ra.end());
        const size_t top = std::min<size_t>(8, cands.size());
        rf.resize(top);
        ra.resize(top);
        for (int round = 0; round < 3; ++round)
            for (size_t j = 0; j < top; ++j) {
                rf[j].first += time_it(cands[rf[j].second], false);
                ra[j].first += time_it(cands[ra[j].second], true);
            }
        std::sort(rf.begin(), rf.end());
        std::sort(ra.begin(), ra.end());
        // among shapes within 6 % of the fastest, prefer one plane of loads
        // in flight, the column orders (z halos, and with groups of columns
        // y halos, from L2), then round robin over the XCDs, then the
        // longest x chunk (fewest halo planes re-read), then the larger
        // column group:
        // that pays when the codec shares the memory system with the step
        // (the sweeps run it beside them)
        auto pick = [&](const std::vector<std::pair<double, size_t>> &r) {
            auto key = [&](size_t j) {
                const fwi_ctx::Shape &h = cands[r[j].second];
                return std::make_tuple(h.deep == 0, h.vz == 2, h.remap >= 2, h.remap != 1, h.xchunk, h.remap);
            };
            size_t k = 0;
            for (size_t j = 1; j < r.size(); ++j)
                if (r[j].first <= 1.06 * r[0].first && key(j) > key(k)) k = j;
            return k;
        };
        const size_t kf = pick(rf), ka = pick(ra);
        const double bf = rf[kf].first / 4, ba = ra[ka].first / 4;
        const fwi_ctx::Shape sf = cands[rf[kf].second], sa = cands[ra[ka].second];
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        c->tuned[ex.grid_key()] = {sf, sa};
        c->drop_graphs();
        out->ncand = (int)cands.size();
        out->fwd_xchunk = sf.xchunk; out->fwd_rows_per_lane = sf.rpl; out->fwd_xcd_order = sf.remap;
        out->adj_xchunk = sa.xchunk; out->adj_rows_per_lane = sa.rpl; out->adj_xcd_order = sa.remap;
        out->fwd_deep = sf.deep;
        out->adj_deep = sa.deep;
        out->fwd_vz = sf.vz;
        out->adj_vz = sa.vz;
        out->fwd_ms = bf;
        out->adj_ms = ba;
        HIPCHK(hipMemsetAsync(c->sb.arena.p, 0, c->sb.arena.n, st));
        HIPCHK(hipStreamSynchronize(st));
    });
}

int fwi_time_shape(fwi_ctx *c, const fwi_grid *g, const float *m, const fwi_shot *shot, const int shape[5],
                   int steps, double *fwd_ms, double *adj_ms, hipStream_t st)
{
    return guarded([&] {
        if (!c || !m || !shape || !fwd_ms || !adj_ms) throw Error{FWI_EINVAL, "null argument"};
        if (steps < 1) throw Error{FWI_EINVAL, "steps must be >= 1"};
        HIPCHK(hipSetDevice(c->device));
        Exec ex{c, make_setup(g, shot, true), st, m, shot};
        const fwi_ctx::Shape sh{shape[0], shape[1], shape[2], shape[3], shape[4]};
        if (!valid_shape(ex.S.ndim, sh)) throw Error{FWI_EINVAL, "invalid launch shape"};
        ensure_fields(&c->sb, ex.S);
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        fill_tuning_fields(c, ex, st);
        *fwd_ms = time_shape(c, ex, shot, sh, false, steps, e0, e1, st);
        *adj_ms = time_shape(c, ex, shot, sh, true, steps, e0, e1, st);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        HIPCHK(hipMemsetAsync(c->sb.arena.p, 0, c->sb.arena.n, st));
        HIPCHK(hipStreamSynchronize(st));
    });
}

int fwi_autotune_batch(fwi_ctx *c, int nshots, const fwi_grid *grids, const float *const *models,
                       const fwi_shot *shots, int steps, fwi_tune_result *out, hipStream_t st)
{
    return guarded([&] {
        if (!c || nshots < 1 || !grids || !models || !shots || !out)
            throw Error{FWI_EINVAL, "null argument or nshots < 1"};
        if (steps < 1) throw Error{FWI_EINVAL, "steps must be >= 1"};
        for (int i = 0; i < nshots; ++i) {
            if (!models[i]) throw Error{FWI_EINVAL, "null model of shot " + std::to_string(i)};
            const fwi_grid &a = grids[0], &b = grids[i];
            if (b.ndim != a.ndim || b.space_order != a.space_order || b.nt != a.nt || b.dt != a.dt)
                throw Error{FWI_EINVAL, "batched shots must share ndim, space order, nt and dt"};
        }
        HIPCHK(hipSetDevice(c->device));
        std::vector<Setup> setups;
        setups.reserve(nshots);
        for (int i = 0; i < nshots; ++i) setups.push_back(make_setup(&grids[i], &shots[i], true));
        while ((int)c->batch.size() < nshots) c->batch.push_back(std::make_unique<ShotBufs>());
        std::vector<Exec> ex;
        ex.reserve(nshots);
        for (int i = 0; i < nshots; ++i) {
            ShotBufs *b = c->batch[i].get();
            ensure_fields(b, setups[i]);
            ex.push_back(Exec{c, setups[i], st, models[i], &shots[i], b});
            // non-zero data in every field the steps read, as fwi_autotune times
            HIPCHK(hipMemsetAsync(b->arena.p, 0, b->arena.n, st));
            ex.back().init_fields();
            for (float *f : {b->fa.p, b->fb.p, b->la.p, b->lb.p, b->gacc.p})
                launch_copy(f, b->coef.p, b->padded_elems, st);
        }
        const int ndim = setups[0].ndim, R = setups[0].R;
        std::vector<int> cands = ndim == 3 ? std::vector<int>{8, 16, 32, 64} : std::vector<int>{4, 8, 16, 32, 64};
        // two launch tables (buffer roles alternate from one launch to the next)
        const size_t tb = ((size_t)nshots * sizeof(BatchEntry) + 255) & ~(size_t)255;
        c->btab.ensure(2 * tb);
        auto table = [&](int xc, bool adj, int parity, BatchEntry *h) {
            int first = 0;
            for (int i = 0; i < nshots; ++i) {
                StepParams p = ex[i].params();
                p.xchunk = xc;
                p.rpl = 2;              // as the batched launches run
                p.vz = 1;
                p.remap = 0;
                p.deep = 0;
                ShotBufs *b = ex[i].B;
                float *a = parity ? b->fb.p : b->fa.p, *o = parity ? b->fa.p : b->fb.p;
                if (adj) {
                    float *l1 = parity ? b->lb.p : b->la.p, *l2 = parity ? b->la.p : b->lb.p;
                    p.u1 = l1; p.u2 = l2; p.out = l2; p.uk = a; p.g = b->gacc.p;
                } else {
                    p.u1 = a; p.u2 = o; p.out = o; p.wav = shots[i].wavelet; p.step = 0;
                }
                h[i] = BatchEntry{};
                h[i].p = p;
                h[i].first = first;
                const int g = step_geometry(h[i], ndim, adj);
                first += ndim == 3 ? (g + 7) & ~7 : g;
            }
            return first;
        };
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        auto time_it = [&](int xc, bool adj) {
            BatchEntry *h[2] = {(BatchEntry *)c->btab.host, (BatchEntry *)(c->btab.host + tb)};
            BatchEntry *d[2] = {(BatchEntry *)c->btab.dev.p, (BatchEntry *)(c->btab.dev.p + tb)};
            const int total = table(xc, adj, 0, h[0]);
            table(xc, adj, 1, h[1]);
            HIPCHK(hipMemcpyAsync(c->btab.dev.p, c->btab.host, 2 * tb, hipMemcpyHostToDevice, st));
            launch_step_batch(d[0], h[0], nshots, total, ndim, R, adj, st);
            HIPCHK(hipEventRecord(e0, st));
            for (int i = 1; i <= steps; ++i) launch_step_batch(d[i & 1], h[i & 1], nshots, total, ndim, R, adj, st);
            HIPCHK(hipEventRecord(e1, st));
            HIPCHK(hipEventSynchronize(e1));     // the host tables are rewritten for the next candidate
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            return (double)ms / steps;
        };
        // every candidate four times, interleaved; the fastest mean, or the
        // longest x chunk within 3 % of it (fewer halo planes re-read)
        std::vector<double> tf(cands.size(), 0.0), ta(cands.size(), 0.0);
        for (int round = 0; round < 4; ++round)
            for (size_t j = 0; j < cands.size(); ++j) {
                tf[j] += time_it(cands[j], false);
                ta[j] += time_it(cands[j], true);
            }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        auto pick = [&](const std::vector<double> &t) {
            size_t best = 0;
            for (size_t j = 1; j < t.size(); ++j)
                if (t[j] < t[best]) best = j;
            size_t k = best;
            for (size_t j = 0; j < t.size(); ++j)
                if (t[j] <= 1.03 * t[best] && cands[j] > cands[k]) k = j;
            return k;
        };
        const size_t kf = pick(tf), ka = pick(ta);
        c->tuned_batch[batch_key(ex)] = {cands[kf], cands[ka]};
        c->drop_graphs();
        for (auto &up : c->batch) {
            if (up->arena.p) HIPCHK(hipMemsetAsync(up->arena.p, 0, up->arena.n, st));
        }
        HIPCHK(hipStreamSynchronize(st));
        *out = fwi_tune_result{};
        out->ncand = (int)cands.size();
        out->fwd_xchunk = cands[kf]; out->fwd_rows_per_lane = 2; out->fwd_xcd_order = 0;
        out->adj_xchunk = cands[ka]; out->adj_rows_per_lane = 2; out->adj_xcd_order = 0;
        out->fwd_ms = tf[kf] / 4;
        out->adj_ms = ta[ka] / 4;
        out->fwd_vz = out->adj_vz = 1;
    });
}

int fwi_bandwidth_probe(const float *const *src, int nsrc, float *const *dst, int ndst, size_t n,
                        int width, int grid, hipStream_t st)
{
    return guarded([&] {
        if (!src || !dst || nsrc < 1 || nsrc > 5 || ndst < 1 || ndst > 2)
            throw Error{FWI_EINVAL, "need 1..5 sources and 1..2 destinations"};
        if (width != 4 && width != 8 && width != 16) throw Error{FWI_EINVAL, "width must be 4, 8 or 16 bytes"};
        if (n % (size_t)(width / 4) != 0) throw Error{FWI_EINVAL, "n must be a multiple of the access width"};
        if (grid < 0 || grid > (1 << 20)) throw Error{FWI_EINVAL, "grid must be in 0..2^20 workgroups"};
        if (grid == 0 && n / (size_t)(width / 4) > ((size_t)1 << 31) * 255)
            throw Error{FWI_EINVAL, "arrays too long for a one-vector-per-lane grid"};
        ProbeArgs a{};
        for (int i = 0; i < nsrc; ++i) {
            if (!src[i] || (uintptr_t)src[i] % (size_t)width) throw Error{FWI_EINVAL, "null or misaligned source"};
            a.src[i] = src[i];
        }
        for (int j = 0; j < ndst; ++j) {
            if (!dst[j] || (uintptr_t)dst[j] % (size_t)width) throw Error{FWI_EINVAL, "null or misaligned destination"};
            a.dst[j] = dst[j];
        }
        a.n = n;
        launch_probe(a, nsrc, ndst, width, grid, st);
        HIPCHK(hipGetLastError());
    });
}

int fwi_revolve_plan(int nsteps, int nslots, fwi_action *out, int cap, int *nactions, long long *nforward)
{
    return guarded([&] {
        if (nsteps < 1 || nslots < 0 || !nactions) throw Error{FWI_EINVAL, "bad arguments"};
        std::vector<fwi_action> a = revolve_plan(nsteps, nslots);
        *nactions = (int)a.size();
        if (nforward) {
            long long f = 0;
            for (auto &x : a)
                if (x.op == FWI_ADVANCE) f += x.b - x.a;
            *nforward = f;
        }
        if ((int)a.size() > cap || !out) throw Error{FWI_ECAPACITY, "action buffer too small"};
        std::copy(a.begin(), a.end(), out);
    });
}

}  // extern "C"
