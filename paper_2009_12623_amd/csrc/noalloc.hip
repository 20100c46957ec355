// Allocation-free checkpoint compression for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc): ckpt_compress with its encode
// workspace (per-chunk bit strings, chunk lengths, tile sums and placement,
// counters, status flags) in one file-scope device array instead of a
// context's buffers.  The kernels are the codec's own; the stream is
// byte for byte the one ckpt_compress writes.
//
// Each GPU the library runs on holds its own copy of the array until the
// process ends.  Its device address is looked up once per device (with
// that device current) and kept; host code passes that address, never the
// symbol, to kernels.  Every call on a GPU shares that GPU's array and it
// keeps the last call's contents, so the counters and flags are cleared at
// the start of each call, and calls that overlap on one GPU race.
#include <cmath>
#include <mutex>
#include <string>

#include "../../include/fwigrad.h"
#include "internal.hpp"

namespace fwi {
namespace {

constexpr size_t STATIC_WORDS = (size_t)4 << 20;    // 32 MiB of u64 words
constexpr int MAX_DEVICES = 64;

__device__ __attribute__((aligned(256))) unsigned long long static_scratch[STATIC_WORDS];

std::mutex g_mu;
unsigned long long *g_ptr[MAX_DEVICES] = {};

// device address of static_scratch on `device` (which must be current)
unsigned long long *scratch_on(int device, std::string &err)
{
    if (device < 0 || device >= MAX_DEVICES) {
        err = "device ordinal beyond the static workspace table";
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(static_scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            err = std::string("hipGetSymbolAddress of the static encode workspace failed: ") +
                  hipGetErrorString(e);
            return nullptr;
        }
        g_ptr[device] = (unsigned long long *)p;
    }
    return g_ptr[device];
}

int fail(int code, const std::string &msg)
{
    set_last_error(msg.c_str());
    return code;
}

}  // namespace
}  // namespace fwi

using namespace fwi;

extern "C" int ckpt_compress_static(const float *field, int ndim, const int n[3], double atol, void *out,
                                    size_t cap, size_t *nbytes, hipStream_t st)
{
    if (!field || !out || !nbytes || !n) return fail(FWI_EINVAL, "null argument");
    if (ndim != 2 && ndim != 3) return fail(FWI_EINVAL, "ndim must be 2 or 3");
    for (int d = 0; d < ndim; ++d)
        if (n[d] < 1) return fail(FWI_EINVAL, "dims must be >= 1");
    if (!(atol >= 2.2250738585072014e-308) || !std::isfinite(atol))
        return fail(FWI_EINVAL, "atol must be a positive normal number");
    FieldView f;
    f.ndim = ndim;
    f.n[0] = n[0];
    f.n[1] = ndim == 3 ? n[1] : 1;
    f.n[2] = ndim == 3 ? n[2] : n[1];
    f.sx = f.n[1] * f.n[2];
    f.sy = ndim == 3 ? f.n[2] : 0;
    f.padded = 0;
    const CodecGeom g = codec_geom(ndim, f.n);
    // chunk words | chunk bit lengths | tile sums + placement | 4 counters | flags
    const size_t ntiles = (size_t)((g.nchunks + 1023) / 1024);
    const size_t words = (size_t)g.nchunks * (size_t)g.max_chunk_words;
    const size_t need = words + (size_t)g.nchunks + (ntiles + 2) + 4 + 1;
    if (need > STATIC_WORDS)
        return fail(FWI_EINVAL, "field needs " + std::to_string(need * 8) +
                                    " bytes of encode workspace, above the static workspace's " +
                                    std::to_string(STATIC_WORDS * 8) + " (use ckpt_compress)");
    int dev = 0;
    hipError_t he = hipGetDevice(&dev);
    if (he != hipSuccess) return fail(FWI_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(he));
    std::string err;
    unsigned long long *base = scratch_on(dev, err);
    if (!base) return fail(FWI_EHIP, err);
    unsigned long long *chunk_bits = base + words;
    unsigned long long *chunk_off = chunk_bits + g.nchunks;
    unsigned long long *misc = chunk_off + ntiles + 2;
    unsigned int *flags = (unsigned int *)(misc + 4);
    // counters and flags start at zero: a fill kernel, not a memset node,
    // so a capturing caller records kernel nodes only
    launch_fill_zero((float *)misc, 10, st);
    EncodeArgs e{};
    e.f = f;
    e.src = field;
    e.atol = atol;
    e.scratch = base;
    e.chunk_bits = chunk_bits;
    e.chunk_off = chunk_off;
    e.dst = (unsigned char *)out;
    e.cap = cap;
    e.out_bytes = misc + 0;
    e.pool_high = misc + 1;
    e.total_bytes = misc + 2;
    e.flags = flags;
    codec_encode(e, st);
    he = hipGetLastError();
    if (he != hipSuccess) return fail(FWI_EHIP, std::string("encode launch: ") + hipGetErrorString(he));
    unsigned long long nb = 0;
    unsigned int fl = 0;
    he = hipMemcpyAsync(&nb, misc, sizeof(nb), hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipMemcpyAsync(&fl, flags, sizeof(fl), hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    if (he != hipSuccess) return fail(FWI_EHIP, std::string("reading the encode status: ") + hipGetErrorString(he));
    if (fl & 1u) return fail(FWI_ENONFINITE, "non-finite value handed to the codec");
    if (fl & 8u) return fail(FWI_ERANGE, "a value at or above atol * 2^23: the fixed-accuracy bound cannot hold");
    if (fl & 2u) return fail(FWI_ECAPACITY, "output buffer smaller than the stream");
    *nbytes = (size_t)nb;
    return FWI_OK;
}
