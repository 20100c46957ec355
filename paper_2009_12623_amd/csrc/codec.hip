// Fixed-accuracy block codec for float32 wavefields (paper Sec. 1.4 and
// Sec. 3: ZFP-style compression of checkpoints at absolute tolerance atol).
//
// Stream (little endian):
//   64-byte header | u64 bit offset per super-chunk of 256 chunks |
//   u32 bit offset per chunk, relative to its super-chunk | pad to 8 bytes |
//   payload: block bit strings, LSB first in u64 words.
// A chunk holds K blocks (16 in 3D, 64 in 2D, halved while the field would
// have fewer than 16384 chunks, down to 1); chunk c = 64 g + l owns the
// blocks g*64K + j*64 + l, j = 0..K-1, so that the 64 lanes of a wave, one
// chunk each, touch 64 neighbouring blocks at every step j.
//
// Per block (4^d values): block exponent emax; skip bit when the block is
// below atol; else exact conversion to int32 at Q = 24 fractional bits,
// a reversible lifting along z, y, x, reorder by total sequency, negabinary,
// then bit planes from the top non-empty one down to P: refinement bits of
// the significant prefix, then either 0 (no new significance) or 1 followed
// by an Elias-gamma code of the extent and the raw bits below its top bit.
//
// GPU mapping: one lane encodes/decodes one chunk, block after block, with
// the whole block in registers.  The 64-coefficient x 32-plane bit matrix is
// turned into plane masks with an in-register 32x32 bit transpose, so every
// per-plane step is a handful of vector instructions and no lane ever waits
// on another.  Encoding writes each chunk to scratch interleaved by lane; a
// tile scan places the chunks and a pack kernel concatenates them at bit
// granularity (each output word is assembled by exactly one thread, and
// consecutive threads assemble consecutive words).  Interior blocks of
// 16-byte-aligned fields are read and written one 16-byte row at a time.
#include <cstring>

#include "internal.hpp"

namespace fwi {

namespace {

constexpr int QB = 24;
typedef float f4v __attribute__((ext_vector_type(4)));

// Every array the codec touches is device (global) memory.  The batched
// kernels take their arguments from job tables in memory, whose pointers the
// compiler cannot tell apart from LDS ones, so it would emit flat accesses;
// on gfx950 those count against the LDS wait counter too, and every wait for
// an LDS read (the scan and pack kernels) would wait for the global loads in
// flight as well.  Accesses made through gp() are global ones.
#define GLOBAL_AS __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ GLOBAL_AS T *gp(T *p)
{
    return (GLOBAL_AS T *)p;
}

// ------------------------------------------------------- sequency tables
template <int D>
struct Seq {
    static constexpr int SZ = D == 3 ? 64 : 16;
    int perm[SZ];
    constexpr Seq() : perm()
    {
        int s = 0;
        for (int tot = 0; tot <= 3 * D; ++tot)
            for (int li = 0; li < SZ; ++li) {
                int ix = D == 3 ? (li >> 4) : (li >> 2);
                int iy = D == 3 ? ((li >> 2) & 3) : 0;
                int iz = li & 3;
                if (ix + iy + iz == tot) perm[s++] = li;
            }
    }
};

template <int D>
struct GeomC {
    static constexpr int SZ = D == 3 ? 64 : 16;
    static constexpr int TP = D == 3 ? 31 : 29;
    static constexpr int G = D == 3 ? 5 : 4;
};

__device__ __forceinline__ int asr1(uint32_t v) { return (int)v >> 1; }

__device__ __forceinline__ void lift_fwd(int &a0, int &a1, int &a2, int &a3)
{
    uint32_t h0 = (uint32_t)a1 - (uint32_t)a0;
    uint32_t l0 = (uint32_t)a0 + (uint32_t)asr1(h0);
    uint32_t h1 = (uint32_t)a3 - (uint32_t)a2;
    uint32_t l1 = (uint32_t)a2 + (uint32_t)asr1(h1);
    uint32_t H = l1 - l0;
    uint32_t L = l0 + (uint32_t)asr1(H);
    h1 -= h0;
    h0 -= (uint32_t)asr1(H);
    a0 = (int)L; a1 = (int)H; a2 = (int)h0; a3 = (int)h1;
}

__device__ __forceinline__ void lift_inv(int &a0, int &a1, int &a2, int &a3)
{
    uint32_t L = a0, H = a1, h0 = a2, h1 = a3;
    h0 += (uint32_t)asr1(H);
    h1 += h0;
    uint32_t l0 = L - (uint32_t)asr1(H);
    uint32_t l1 = H + l0;
    uint32_t x0 = l0 - (uint32_t)asr1(h0);
    uint32_t x1 = h0 + x0;
    uint32_t x2 = l1 - (uint32_t)asr1(h1);
    uint32_t x3 = h1 + x2;
    a0 = (int)x0; a1 = (int)x1; a2 = (int)x2; a3 = (int)x3;
}

template <int D>
__device__ __forceinline__ void block_fwd(int *c)
{
    if (D == 3) {
#pragma unroll
        for (int i = 0; i < 16; ++i) lift_fwd(c[4 * i], c[4 * i + 1], c[4 * i + 2], c[4 * i + 3]);
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int z = 0; z < 4; ++z) {
                int b = 16 * x + z;
                lift_fwd(c[b], c[b + 4], c[b + 8], c[b + 12]);
            }
#pragma unroll
        for (int i = 0; i < 16; ++i) lift_fwd(c[i], c[i + 16], c[i + 32], c[i + 48]);
    } else {
#pragma unroll
        for (int x = 0; x < 4; ++x) lift_fwd(c[4 * x], c[4 * x + 1], c[4 * x + 2], c[4 * x + 3]);
#pragma unroll
        for (int z = 0; z < 4; ++z) lift_fwd(c[z], c[z + 4], c[z + 8], c[z + 12]);
    }
}

template <int D>
__device__ __forceinline__ void block_inv(int *c)
{
    if (D == 3) {
#pragma unroll
        for (int i = 0; i < 16; ++i) lift_inv(c[i], c[i + 16], c[i + 32], c[i + 48]);
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int z = 0; z < 4; ++z) {
                int b = 16 * x + z;
                lift_inv(c[b], c[b + 4], c[b + 8], c[b + 12]);
            }
#pragma unroll
        for (int i = 0; i < 16; ++i) lift_inv(c[4 * i], c[4 * i + 1], c[4 * i + 2], c[4 * i + 3]);
    } else {
#pragma unroll
        for (int z = 0; z < 4; ++z) lift_inv(c[z], c[z + 4], c[z + 8], c[z + 12]);
#pragma unroll
        for (int x = 0; x < 4; ++x) lift_inv(c[4 * x], c[4 * x + 1], c[4 * x + 2], c[4 * x + 3]);
    }
}

// 32x32 bit-matrix transpose in place: afterwards bit c of a[r] is the
// former bit r of a[c].  Five rounds of block swaps.
__device__ __forceinline__ void transpose32(uint32_t *a)
{
#pragma unroll
    for (int j = 16, round = 0; round < 5; j >>= 1, ++round) {
        const uint32_t m = j == 16 ? 0x0000FFFFu : j == 8 ? 0x00FF00FFu : j == 4 ? 0x0F0F0F0Fu
                         : j == 2 ? 0x33333333u : 0x55555555u;
#pragma unroll
        for (int k = 0; k < 32; ++k) {
            if (k & j) continue;
            uint32_t t = ((a[k] >> j) ^ a[k + j]) & m;
            a[k] ^= t << j;
            a[k + j] ^= t;
        }
    }
}

__device__ __forceinline__ uint32_t lowmask32(int n)
{
    return n >= 32 ? 0xFFFFFFFFu : ((1u << n) - 1u);
}

__device__ __forceinline__ unsigned long long lowmask64(int n)
{
    return n >= 64 ? ~0ull : ((1ull << n) - 1ull);
}

// Chunk scratch is interleaved by lane: word w of chunk c lives at
// scratch[(c / 64) * 64 * chunk_words + w * 64 + c % 64], so the 64 lanes of a
// wave writing their w-th words touch one 512-byte span.
__host__ __device__ __forceinline__ long scratch_word(long c, long w, long chunk_words)
{
    return (c >> 6) * 64 * chunk_words + w * 64 + (c & 63);
}

struct BitWriter {
    unsigned long long acc;
    int fill;
    GLOBAL_AS unsigned long long *out;   // word 0 of this lane; word w at out[64 w]
    long w;
    __device__ __forceinline__ void put(uint32_t v, int n)    // v < 2^n, n <= 32
    {
        if (n <= 0) return;
        acc |= (unsigned long long)v << fill;
        fill += n;
        if (fill >= 64) {
            out[64 * w++] = acc;
            fill -= 64;
            acc = fill ? ((unsigned long long)v >> (n - fill)) : 0ull;
        }
    }
    __device__ __forceinline__ void put64(unsigned long long v, int n)   // v < 2^n, n <= 64
    {
        if (n > 32) {
            put((uint32_t)v, 32);
            put((uint32_t)(v >> 32), n - 32);
        } else {
            put((uint32_t)v, n);
        }
    }
};

struct BitReader {
    const GLOBAL_AS unsigned long long *w;
    long nw;
    long idx;                       // word index of lo
    unsigned long long lo, hi;
    unsigned long long nx;          // word idx + 2, loaded ahead of its use
    unsigned long long pos;         // absolute bit position
    __device__ __forceinline__ unsigned long long ld(long i) const { return i < nw && i >= 0 ? w[i] : 0ull; }
    __device__ __forceinline__ void seek(unsigned long long p)
    {
        pos = p;
        idx = (long)(p >> 6);
        lo = ld(idx);
        hi = ld(idx + 1);
        nx = ld(idx + 2);
    }
    __device__ __forceinline__ uint32_t peek32() const
    {
        int sh = (int)(pos & 63);
        unsigned long long v = sh ? ((lo >> sh) | (hi << (64 - sh))) : lo;
        return (uint32_t)v;
    }
    __device__ __forceinline__ void skip(int n)
    {
        pos += (unsigned long long)n;
        long ni = (long)(pos >> 6);
        if (ni != idx) {
            if (ni == idx + 1) {
                lo = hi;
                hi = nx;
            } else {
                lo = ld(ni);
                hi = ld(ni + 1);
            }
            nx = ld(ni + 2);
            idx = ni;
        }
    }
    __device__ __forceinline__ uint32_t get(int n)     // n <= 32
    {
        if (n <= 0) return 0u;
        uint32_t v = peek32() & lowmask32(n);
        skip(n);
        return v;
    }
    __device__ __forceinline__ unsigned long long get64(int n)
    {
        if (n > 32) {
            unsigned long long a = get(32);
            return a | ((unsigned long long)get(n - 32) << 32);
        }
        return get(n);
    }
};

__device__ __forceinline__ long chunk_block(long c, int j, int K, long nblocks)
{
    long b = (c >> 6) * 64L * K + (long)j * 64 + (c & 63);
    return b < nblocks ? b : -1;
}

__device__ __forceinline__ void block_coords(long b, const long *nb, long &bx, long &by, long &bz)
{
    bz = b % nb[2];
    long r = b / nb[2];
    by = r % nb[1];
    bx = r / nb[1];
}

// ------------------------------------------------------------------ encode
// arguments of the per-chunk encode and decode (one field)
struct EncodeK {
    FieldView f;
    const float *src;
    long nb0, nb1, nb2, nblocks, nchunks;
    int kblk, minexp, vec;
    unsigned long long *scratch;
    long chunk_words;
    unsigned long long *chunk_bits;
    unsigned int *flags;
};

struct DecodeK {
    FieldView f;
    float *dst;
    const unsigned char *stream, *pool;
    const StreamSlot *slots;
    int slot_index;
    long nb0, nb1, nb2, nblocks, nchunks;
    int kblk;
    long nsuper, table_bytes;
    unsigned int *flags;
    int vec;
};

template <int D>
__device__ __forceinline__ void encode_body(const EncodeK &k, long blk)
{
    using GC = GeomC<D>;
    constexpr int SZ = GC::SZ;
    constexpr Seq<D> seq{};
    const FieldView &f = k.f;
    const GLOBAL_AS float *src = gp(k.src);
    const long nb0 = k.nb0, nb1 = k.nb1, nb2 = k.nb2, nblocks = k.nblocks, nchunks = k.nchunks;
    const int kblk = k.kblk, minexp = k.minexp, vec = k.vec;
    unsigned long long *scratch = k.scratch;
    const long chunk_words = k.chunk_words;
    unsigned long long *chunk_bits = k.chunk_bits;
    unsigned int *flags = k.flags;
    const long c = blk * 64 + threadIdx.x;
    if (c >= nchunks) return;
    const long nb[3] = {nb0, nb1, nb2};
    BitWriter bw{0ull, 0, gp(scratch) + scratch_word(c, 0, chunk_words), 0};
    bool nonfinite = false, outrange = false;
    // padded fields: the rows of the next block are loaded while the current
    // one is coded
    f4v pf[SZ / 4];
    auto load_rows = [&](long bb) {
        long qx, qy, qz;
        block_coords(bb, nb, qx, qy, qz);
#pragma unroll
        for (int r = 0; r < SZ / 4; ++r) {
            const int ix = D == 3 ? (r >> 2) : r;
            const int iy = D == 3 ? (r & 3) : 0;
            long x = 4 * qx + ix, y = 4 * qy + iy;
            x = x < f.n[0] ? x : f.n[0] - 1;
            y = y < f.n[1] ? y : f.n[1] - 1;
            pf[r] = __builtin_nontemporal_load((const GLOBAL_AS f4v *)(src + x * f.sx + y * f.sy + 4 * qz));
        }
    };
    if (vec == 2) {
        const long b0 = chunk_block(c, 0, kblk, nblocks);
        if (b0 >= 0) load_rows(b0);
    }
    for (int j = 0; j < kblk; ++j) {
        const long b = chunk_block(c, j, kblk, nblocks);
        if (b < 0) break;
        long bx, by, bz;
        block_coords(b, nb, bx, by, bz);
        uint32_t w[SZ];
        const bool inner = vec && 4 * bx + 3 < f.n[0] && (D == 2 || 4 * by + 3 < f.n[1]) && 4 * bz + 3 < f.n[2];
        if (vec == 2) {
            // padded field: one 16-byte load per row for every block; rows
            // past the end repeat the last row, and the z tail repeats the
            // last valid sample (the extra values read are padding)
            const long zl = f.n[2] - 1 - 4 * bz;             // last valid z in the block (>= 0)
            f4v cur[SZ / 4];
#pragma unroll
            for (int r = 0; r < SZ / 4; ++r) cur[r] = pf[r];
            const long bn = j + 1 < kblk ? chunk_block(c, j + 1, kblk, nblocks) : -1;
            if (bn >= 0) load_rows(bn);
#pragma unroll
            for (int r = 0; r < SZ / 4; ++r) {
                const f4v v = cur[r];
                const float e1 = zl >= 1 ? v.y : v.x;
                const float e2 = zl >= 2 ? v.z : e1;
                const float e3 = zl >= 3 ? v.w : e2;
                w[4 * r + 0] = __float_as_uint(v.x);
                w[4 * r + 1] = __float_as_uint(e1);
                w[4 * r + 2] = __float_as_uint(e2);
                w[4 * r + 3] = __float_as_uint(e3);
            }
        } else if (inner) {
            // whole block inside: one 16-byte load per (x, y) row
#pragma unroll
            for (int r = 0; r < SZ / 4; ++r) {
                const int ix = D == 3 ? (r >> 2) : r;
                const int iy = D == 3 ? (r & 3) : 0;
                const f4v v = __builtin_nontemporal_load(
                    (const GLOBAL_AS f4v *)(src + (4 * bx + ix) * f.sx + (4 * by + iy) * f.sy + 4 * bz));
                w[4 * r + 0] = __float_as_uint(v.x);
                w[4 * r + 1] = __float_as_uint(v.y);
                w[4 * r + 2] = __float_as_uint(v.z);
                w[4 * r + 3] = __float_as_uint(v.w);
            }
        } else {
            // partial block: repeat the last valid sample along each axis
#pragma unroll
            for (int li = 0; li < SZ; ++li) {
                const int ix = D == 3 ? (li >> 4) : (li >> 2);
                const int iy = D == 3 ? ((li >> 2) & 3) : 0;
                const int iz = li & 3;
                long x = 4 * bx + ix, y = 4 * by + iy, z = 4 * bz + iz;
                x = x < f.n[0] ? x : f.n[0] - 1;
                y = y < f.n[1] ? y : f.n[1] - 1;
                z = z < f.n[2] ? z : f.n[2] - 1;
                w[li] = __float_as_uint(src[x * f.sx + y * f.sy + z]);
            }
        }
        int Emax = 0;
#pragma unroll
        for (int li = 0; li < SZ; ++li) {
            const int E = (int)((w[li] >> 23) & 0xFFu);
            nonfinite |= (E == 0xFF);
            Emax = E > Emax ? E : Emax;
        }
        const int emax = Emax - 126;
        if (Emax == 0 || emax <= minexp) {
            bw.put(0u, 1);
            continue;
        }
        // fixed-accuracy bound needs emax <= minexp + Q - 1 (|x| < atol 2^23)
        outrange |= emax > minexp + QB - 1;
        int ci[SZ];
#pragma unroll
        for (int li = 0; li < SZ; ++li) {
            const int E = (int)((w[li] >> 23) & 0xFFu);
            const uint32_t mant = (w[li] & 0x7FFFFFu) | 0x800000u;
            const int sh = Emax - E;
            uint32_t mag = sh >= 32 ? 0u : (mant >> sh);
            mag = E == 0 ? 0u : mag;
            ci[li] = (w[li] >> 31) ? -(int)mag : (int)mag;
        }
        block_fwd<D>(ci);
        uint32_t lo[32], hi[32];
#pragma unroll
        for (int s = 0; s < 32; ++s) {
            lo[s] = s < SZ ? (((uint32_t)ci[seq.perm[s]] + 0xAAAAAAAAu) ^ 0xAAAAAAAAu) : 0u;
            hi[s] = (D == 3) ? (((uint32_t)ci[seq.perm[32 + (s & 31)]] + 0xAAAAAAAAu) ^ 0xAAAAAAAAu) : 0u;
        }
        transpose32(lo);
        if (D == 3) transpose32(hi);
        int P = minexp - emax + QB - GC::G;
        P = P < 0 ? 0 : P;
        int fp = -1;
#pragma unroll
        for (int p = 0; p < 32; ++p)
            if (p >= P && (lo[p] | hi[p])) fp = p;
        const int zs = (fp < 0 || GC::TP - fp > 7) ? 7 : GC::TP - fp;
        const int S = GC::TP - zs;
        bw.put(1u, 1);
        bw.put((uint32_t)(emax + 127), 8);
        bw.put((uint32_t)zs, 3);
        int n = 0;
#pragma unroll
        for (int p = 31; p >= 0; --p) {
            if (p > S || p < P) continue;
            const unsigned long long xp = ((unsigned long long)hi[p] << 32) | lo[p];
            bw.put64(xp & lowmask64(n), n);
            if (n < SZ) {
                const unsigned long long xr = xp >> n;
                if (xr == 0ull) {
                    bw.put(0u, 1);
                } else {
                    const int t = 63 - __clzll((long long)xr);
                    const uint32_t v = (uint32_t)t + 1u;
                    const int L = 31 - __clz((int)v);
                    // 1, then L zeros, a one and the L low bits of v
                    bw.put(1u, 1);
                    bw.put((1u << L) | ((v & lowmask32(L)) << (L + 1)), 2 * L + 1);
                    bw.put64(xr & lowmask64(t), t);
                    n += t + 1;
                }
            }
        }
    }
    if (bw.fill) bw.out[64 * bw.w] = bw.acc;
    gp(chunk_bits)[c] = (unsigned long long)bw.w * 64ull + (unsigned long long)bw.fill;
    if (nonfinite) atomicOr(flags, 1u);
    if (outrange) atomicOr(flags, 8u);
}

// --------------------------------------------------------------- placement
constexpr int TILE = 1024;

__device__ __forceinline__ void tile_sum_body(const unsigned long long *chunk_bits, long nchunks,
                                              unsigned long long *tile_sum, long blk)
{
    __shared__ unsigned long long red[TILE];
    const long c = blk * TILE + threadIdx.x;
    red[threadIdx.x] = c < nchunks ? gp(chunk_bits)[c] : 0ull;
    __syncthreads();
    for (int s = TILE / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) gp(tile_sum)[blk] = red[0];
}

struct PlanArgs {
    int ndim;
    unsigned int dims[3];
    double atol;
    int minexp, guard, tp, log2k;
    long nblocks, nchunks, nsuper;
    long table_bytes;
    int ntiles;
    unsigned long long *tile_sum;     // in: sums, out: exclusive prefix
    unsigned char *dst;               // fixed destination or nullptr
    unsigned long long cap;
    unsigned char *pool;
    unsigned long long pool_cap;
    StreamSlot *slots;
    int slot_index, prev_index;
    unsigned long long *out_bytes;
    unsigned long long *dst_offset;   // device scratch: byte offset of dst in pool (or 0)
    unsigned int *flags;
    unsigned long long *pool_high;
    unsigned long long *total_bytes;
};

__device__ __forceinline__ void st64(unsigned char *p, unsigned long long v)
{
    for (int i = 0; i < 8; ++i) gp(p)[i] = (unsigned char)(v >> (8 * i));
}

__device__ __forceinline__ void st32(unsigned char *p, unsigned int v)
{
    for (int i = 0; i < 4; ++i) gp(p)[i] = (unsigned char)(v >> (8 * i));
}

__device__ __forceinline__ void plan_body(const PlanArgs &a)
{
    __shared__ unsigned long long sc[256];
    __shared__ unsigned long long carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < a.ntiles; base += 256) {
        const int t = base + threadIdx.x;
        unsigned long long v = t < a.ntiles ? a.tile_sum[t] : 0ull;
        sc[threadIdx.x] = v;
        __syncthreads();
        for (int s = 1; s < 256; s <<= 1) {
            unsigned long long add = (int)threadIdx.x >= s ? sc[threadIdx.x - s] : 0ull;
            __syncthreads();
            sc[threadIdx.x] += add;
            __syncthreads();
        }
        if (t < a.ntiles) a.tile_sum[t] = carry + sc[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 255) carry += sc[255];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const unsigned long long total_bits = carry;
    const unsigned long long bytes = 64ull + (unsigned long long)a.table_bytes + 8ull * ((total_bits + 63ull) / 64ull);
    *a.out_bytes = bytes;
    *a.total_bytes += bytes;
    unsigned char *dst = a.dst;
    unsigned long long off = 0;
    bool ok = true;
    if (dst) {
        ok = bytes <= a.cap;
    } else {
        unsigned long long start = 0;
        if (a.prev_index >= 0) {
            const StreamSlot &p = a.slots[a.prev_index];
            start = (p.offset + p.bytes + 255ull) & ~255ull;
        }
        off = start;
        // 8 bytes of slack so readers may fetch one word past the end
        ok = start + bytes + 8ull <= a.pool_cap;
        StreamSlot s;
        s.offset = start;
        s.bytes = ok ? bytes : 0ull;
        s.valid = ok ? 1 : 0;
        s.pad = 0;
        a.slots[a.slot_index] = s;
        if (ok) {
            dst = a.pool + start;
            unsigned long long end = start + bytes;
            if (end > *a.pool_high) *a.pool_high = end;
        }
    }
    *a.dst_offset = off;
    if (!ok) {
        atomicOr(a.flags, 2u);
        return;
    }
    // header
    unsigned char *h = dst;
    h[0] = 'F'; h[1] = 'W'; h[2] = 'Z'; h[3] = '1';
    h[4] = 1; h[5] = 0; h[6] = (unsigned char)a.ndim; h[7] = QB;
    st32(h + 8, a.dims[0]); st32(h + 12, a.dims[1]); st32(h + 16, a.dims[2]);
    h[20] = (unsigned char)a.guard; h[21] = (unsigned char)a.log2k;
    h[22] = (unsigned char)a.tp; h[23] = 0;
    st64(h + 24, (unsigned long long)__double_as_longlong(a.atol));
    st32(h + 32, (unsigned int)a.minexp);
    st32(h + 36, (unsigned int)a.nchunks);
    st64(h + 40, (unsigned long long)a.nblocks);
    st64(h + 48, total_bits);
    st64(h + 56, bytes);
}

struct PackArgs {
    const unsigned long long *scratch;
    long chunk_words;
    const unsigned long long *chunk_bits;
    long nchunks, nsuper;
    long table_bytes;
    const unsigned long long *tile_prefix;
    unsigned char *dst;          // fixed destination, or nullptr (pool + *dst_offset)
    unsigned char *pool;
    const unsigned long long *dst_offset;
    const unsigned int *flags;
};

__device__ __forceinline__ void pack_body(const PackArgs &a, long blk)
{
    __shared__ unsigned long long sc[TILE];
    if (*gp(a.flags) & 2u) return;
    unsigned char *dst = a.dst ? a.dst : a.pool + *gp(a.dst_offset);
    const GLOBAL_AS unsigned long long *chunk_bits = gp(a.chunk_bits);
    const GLOBAL_AS unsigned long long *scratch = gp(a.scratch);
    const GLOBAL_AS unsigned long long *tile_prefix = gp(a.tile_prefix);
    const long c = blk * TILE + threadIdx.x;
    const unsigned long long len = c < a.nchunks ? chunk_bits[c] : 0ull;
    sc[threadIdx.x] = len;
    __syncthreads();
    for (int s = 1; s < TILE; s <<= 1) {
        unsigned long long add = (int)threadIdx.x >= s ? sc[threadIdx.x - s] : 0ull;
        __syncthreads();
        sc[threadIdx.x] += add;
        __syncthreads();
    }
    if (c < a.nchunks) {
        const unsigned long long off = tile_prefix[blk] + sc[threadIdx.x] - len;
        // tables: super-chunk base (the first chunk of each super-chunk) and
        // relative chunk offsets (a super-chunk of 256 lies inside one tile)
        unsigned char *tab = dst + 64;
        const long sup0 = (c / 256) * 256 - blk * TILE;   // in-tile index of the super-chunk head
        const unsigned long long head = tile_prefix[blk] + (sup0 > 0 ? sc[sup0 - 1] : 0ull);
        if ((c & 255) == 0) st64(tab + 8 * (c / 256), off);
        st32(tab + 8 * a.nsuper + 4 * c, (unsigned int)(off - head));
    }
    // payload: the block writes every word whose first bit lies in this
    // tile; consecutive threads take consecutive words (coalesced reads of
    // the chunk scratch and coalesced writes), finding the chunk that holds
    // the word's first bit by binary search over the tile's prefix sums
    __syncthreads();
    GLOBAL_AS unsigned long long *out = gp((unsigned long long *)(dst + 64 + a.table_bytes));
    const unsigned long long base = tile_prefix[blk];
    const unsigned long long tile_end = base + sc[TILE - 1];
    const long c0 = blk * TILE;
    for (unsigned long long w = ((base + 63ull) >> 6) + threadIdx.x; (w << 6) < tile_end; w += TILE) {
        unsigned long long pos = w << 6;
        int lo = 0, hi = TILE - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (base + sc[mid] > pos) hi = mid;
            else lo = mid + 1;
        }
        long cc = c0 + lo;
        unsigned long long cstart = base + (lo ? sc[lo - 1] : 0ull);
        unsigned long long clen = sc[lo] - (lo ? sc[lo - 1] : 0ull);
        unsigned long long word = 0ull;
        int got = 0;
        while (got < 64) {
            if (pos >= cstart + clen) {
                // next chunk (possibly in the next tile)
                ++cc;
                if (cc >= a.nchunks) break;
                cstart += clen;
                clen = chunk_bits[cc];
                continue;
            }
            const unsigned long long lb = pos - cstart;       // local bit in chunk cc
            const int sh = (int)(lb & 63);
            unsigned long long v = scratch[scratch_word(cc, (long)(lb >> 6), a.chunk_words)] >> sh;
            int avail = 64 - sh;
            if ((unsigned long long)avail > clen - lb) avail = (int)(clen - lb);
            const int take = avail < 64 - got ? avail : 64 - got;
            v &= lowmask64(take);
            word |= v << got;
            got += take;
            pos += (unsigned long long)take;
        }
        out[w] = word;
    }
}

// ------------------------------------------------------------------ decode
// absolute payload bit where chunk c starts (super-chunk base + relative offset)
__device__ __forceinline__ unsigned long long chunk_start(const GLOBAL_AS unsigned char *s, long nsuper, long c)
{
    unsigned long long sup = 0;
    unsigned int rel = 0;
    for (int i = 0; i < 8; ++i) sup |= (unsigned long long)s[64 + 8 * (c / 256) + i] << (8 * i);
    for (int i = 0; i < 4; ++i) rel |= (unsigned int)s[64 + 8 * nsuper + 4 * c + i] << (8 * i);
    return sup + rel;
}

template <int D>
__device__ __forceinline__ void decode_body(const DecodeK &k, long blk)
{
    using GC = GeomC<D>;
    constexpr int SZ = GC::SZ;
    constexpr Seq<D> seq{};
    const FieldView &f = k.f;
    float *dst = k.dst;
    const unsigned char *stream = k.stream, *pool = k.pool;
    const StreamSlot *slots = k.slots;
    const int slot_index = k.slot_index;
    const long nb0 = k.nb0, nb1 = k.nb1, nb2 = k.nb2, nblocks = k.nblocks, nchunks = k.nchunks;
    const int kblk = k.kblk;
    const long nsuper = k.nsuper, table_bytes = k.table_bytes;
    unsigned int *flags = k.flags;
    const int vec = k.vec;
    const long c = blk * 64 + threadIdx.x;
    if (c >= nchunks) return;
    const GLOBAL_AS unsigned char *s = gp(stream);
    if (!stream) {
        const GLOBAL_AS StreamSlot *sl = gp(slots) + slot_index;
        if (!sl->valid) return;
        s = gp(pool) + sl->offset;
    }
    const long nb[3] = {nb0, nb1, nb2};
    unsigned long long pbits = 0;
    for (int i = 0; i < 8; ++i) pbits |= (unsigned long long)s[48 + i] << (8 * i);
    const unsigned long long start = chunk_start(s, nsuper, c);
    const int minexp = (int)((unsigned int)s[32] | ((unsigned int)s[33] << 8) |
                             ((unsigned int)s[34] << 16) | ((unsigned int)s[35] << 24));
    BitReader br;
    br.w = (const GLOBAL_AS unsigned long long *)(s + 64 + table_bytes);
    br.nw = (long)((pbits + 63) / 64);
    br.seek(start);
    for (int j = 0; j < kblk; ++j) {
        const long b = chunk_block(c, j, kblk, nblocks);
        if (b < 0) break;
        // integer coefficients of the block (all zero for a skipped block);
        // the float values are formed as they are stored
        int ci[SZ];
        int emax = 0;
        if (br.pos >= pbits) { atomicOr(flags, 4u); return; }
        if (!br.get(1)) {
#pragma unroll
            for (int li = 0; li < SZ; ++li) ci[li] = 0;
        } else {
            emax = (int)br.get(8) - 127;
            const int zs = (int)br.get(3);
            const int S = GC::TP - zs;
            int P = minexp - emax + QB - GC::G;
            P = P < 0 ? 0 : P;
            uint32_t lo[32], hi[32];
            int n = 0;
            bool bad = false;
#pragma unroll
            for (int p = 31; p >= 0; --p) {
                lo[p] = 0u;
                hi[p] = 0u;
                if (p > S || p < P || bad) continue;
                unsigned long long xp = br.get64(n);
                if (n < SZ && br.get(1)) {
                    const uint32_t pk = br.peek32();
                    const int L = pk ? __ffs((int)pk) - 1 : 32;
                    if (L > 6) { bad = true; continue; }
                    br.skip(L + 1);
                    const int t = (int)(((1u << L) | br.get(L)) - 1u);
                    if (t > SZ - 1 - n) { bad = true; continue; }
                    const unsigned long long raw = br.get64(t);
                    xp |= ((1ull << t) | raw) << n;
                    n += t + 1;
                }
                lo[p] = (uint32_t)xp;
                hi[p] = (uint32_t)(xp >> 32);
            }
            if (bad || br.pos > pbits) { atomicOr(flags, 4u); return; }
            transpose32(lo);
            if (D == 3) transpose32(hi);
#pragma unroll
            for (int s2 = 0; s2 < SZ; ++s2) {
                const uint32_t u = s2 < 32 ? lo[s2] : hi[s2 & 31];
                ci[seq.perm[s2]] = (int)((u ^ 0xAAAAAAAAu) - 0xAAAAAAAAu);
            }
            block_inv<D>(ci);
        }
        // int32 -> float32 (round to nearest even), scaled by 2^(emax - Q)
        // through the exponent field; below 2^-126 -> +0, overflow saturates
        auto val = [&](int li) {
            const float r = ldexpf((float)ci[li], emax - QB);
            const float a = fabsf(r);
            float o = a < 1.17549435e-38f ? 0.0f : r;
            return a > 3.40282347e38f ? copysignf(3.40282347e38f, r) : o;
        };
        long bx, by, bz;
        block_coords(b, nb, bx, by, bz);
        if (vec == 2) {
            // padded field: whole-block row stores; entries past the field's
            // end are written as zero (they are padding, which stays zero)
            const long zl = f.n[2] - 1 - 4 * bz;
#pragma unroll
            for (int r = 0; r < SZ / 4; ++r) {
                const int ix = D == 3 ? (r >> 2) : r;
                const int iy = D == 3 ? (r & 3) : 0;
                const long x = 4 * bx + ix, y = 4 * by + iy;
                const bool row = x < f.n[0] && y < f.n[1];
                f4v v;
                v.x = row ? val(4 * r) : 0.0f;
                v.y = row && zl >= 1 ? val(4 * r + 1) : 0.0f;
                v.z = row && zl >= 2 ? val(4 * r + 2) : 0.0f;
                v.w = row && zl >= 3 ? val(4 * r + 3) : 0.0f;
                // 3D working fields are far larger than the caches and are
                // read by the next stencil step: stream them out
                if (D == 3) __builtin_nontemporal_store(v, (GLOBAL_AS f4v *)(gp(dst) + x * f.sx + y * f.sy + 4 * bz));
                else *(GLOBAL_AS f4v *)(gp(dst) + x * f.sx + y * f.sy + 4 * bz) = v;
            }
        } else if (vec && 4 * bx + 3 < f.n[0] && (D == 2 || 4 * by + 3 < f.n[1]) && 4 * bz + 3 < f.n[2]) {
            // whole block inside: one 16-byte store per (x, y) row
#pragma unroll
            for (int r = 0; r < SZ / 4; ++r) {
                const int ix = D == 3 ? (r >> 2) : r;
                const int iy = D == 3 ? (r & 3) : 0;
                f4v v;
                v.x = val(4 * r);
                v.y = val(4 * r + 1);
                v.z = val(4 * r + 2);
                v.w = val(4 * r + 3);
                *(GLOBAL_AS f4v *)(gp(dst) + (4 * bx + ix) * f.sx + (4 * by + iy) * f.sy + 4 * bz) = v;
            }
        } else {
#pragma unroll
            for (int li = 0; li < SZ; ++li) {
                const int ix = D == 3 ? (li >> 4) : (li >> 2);
                const int iy = D == 3 ? ((li >> 2) & 3) : 0;
                const int iz = li & 3;
                const long x = 4 * bx + ix, y = 4 * by + iy, z = 4 * bz + iz;
                if (x < f.n[0] && y < f.n[1] && z < f.n[2]) gp(dst)[x * f.sx + y * f.sy + z] = val(li);
            }
        }
    }
}

int minexp_of(double atol)
{
    unsigned long long bits;
    memcpy(&bits, &atol, 8);
    return (int)((bits >> 52) & 0x7FF) - 1023;
}

}  // namespace

CodecGeom codec_geom(int ndim, const long n[3])
{
    CodecGeom g;
    g.ndim = ndim;
    g.nblocks = 1;
    for (int d = 0; d < 3; ++d) {
        g.nb[d] = (n[d] + 3) / 4;
        g.nblocks *= g.nb[d];
    }
    // K blocks per chunk: 16 (3D) / 64 (2D), halved while the field would
    // have fewer than 16384 chunks (one lane each), down to 1
    g.kblk = ndim == 3 ? 16 : 64;
    while (g.kblk > 1 && (g.nblocks + g.kblk - 1) / g.kblk < 16384) g.kblk >>= 1;
    g.size = ndim == 3 ? 64 : 16;
    g.tp = ndim == 3 ? 31 : 29;
    g.guard = ndim == 3 ? 5 : 4;
    const long per_group = 64L * g.kblk;
    g.nchunks = 64L * ((g.nblocks + per_group - 1) / per_group);
    g.nsuper = (g.nchunks + 255) / 256;
    g.table_bytes = ((8 * g.nsuper + 4 * g.nchunks) + 7) & ~7L;
    const int lg = ndim == 3 ? 6 : 4;
    const long block_bits = 12 + (long)(g.tp + 1) * (g.size + 1 + 2 * lg);
    g.max_chunk_words = (g.kblk * block_bits + 63) / 64;
    return g;
}

long codec_bound(const CodecGeom &g)
{
    const int lg = g.ndim == 3 ? 6 : 4;
    const long block_bits = 12 + (long)(g.tp + 1) * (g.size + 1 + 2 * lg);
    return 64 + g.table_bytes + 8 * ((g.nblocks * block_bits + 63) / 64);
}

// Encode pipeline: encode (lane per chunk) -> tile sums -> plan (placement,
// header) -> pack (tables + payload).  Scratch layout: scratch words
// (nchunks * max_chunk_words), chunk_bits (nchunks), tile sums.
// 16-byte row accesses are valid when every block row starts 16-byte
// aligned (1); whole blocks may be read and written when the field also
// sits in the zero-padded layout (2)
static int rows_vectorizable(const FieldView &f, const float *p)
{
    const bool aligned = ((uintptr_t)p % 16 == 0) && f.sx % 4 == 0 && (f.ndim == 2 || f.sy % 4 == 0);
    return aligned ? (f.padded ? 2 : 1) : 0;
}

// one field's encode pipeline: encode -> tile sums -> placement -> pack
struct EncJob {
    EncodeK enc;
    PlanArgs plan;
    PackArgs pack;
    int wave0, tile0;          // first encode wave / first tile in a batched launch
};

struct DecJob {
    DecodeK dec;
    int wave0;
};

static EncJob make_enc_job(const EncodeArgs &e)
{
    const CodecGeom g = codec_geom(e.f.ndim, e.f.n);
    const int minexp = minexp_of(e.atol);
    const int ntiles = (int)((g.nchunks + TILE - 1) / TILE);
    EncJob j{};
    EncodeK &k = j.enc;
    k.f = e.f;
    k.src = e.src;
    k.nb0 = g.nb[0]; k.nb1 = g.nb[1]; k.nb2 = g.nb[2];
    k.nblocks = g.nblocks;
    k.nchunks = g.nchunks;
    k.kblk = g.kblk;
    k.minexp = minexp;
    k.vec = rows_vectorizable(e.f, e.src);
    k.scratch = e.scratch;
    k.chunk_words = g.max_chunk_words;
    k.chunk_bits = e.chunk_bits;
    k.flags = e.flags;
    unsigned long long *tile = e.chunk_off;   // ntiles sums, then the pool offset
    PlanArgs &pa = j.plan;
    pa.ndim = e.f.ndim;
    if (e.f.ndim == 3) {
        pa.dims[0] = (unsigned)e.f.n[0]; pa.dims[1] = (unsigned)e.f.n[1]; pa.dims[2] = (unsigned)e.f.n[2];
    } else {
        pa.dims[0] = (unsigned)e.f.n[0]; pa.dims[1] = (unsigned)e.f.n[2]; pa.dims[2] = 1u;
    }
    pa.atol = e.atol;
    pa.minexp = minexp;
    pa.guard = g.guard;
    pa.tp = g.tp;
    pa.log2k = __builtin_ctz((unsigned)g.kblk);    // blocks per chunk
    pa.nblocks = g.nblocks;
    pa.nchunks = g.nchunks;
    pa.nsuper = g.nsuper;
    pa.table_bytes = g.table_bytes;
    pa.ntiles = ntiles;
    pa.tile_sum = tile;
    pa.dst = e.dst;
    pa.cap = e.cap;
    pa.pool = e.pool;
    pa.pool_cap = e.pool_cap;
    pa.slots = e.slots;
    pa.slot_index = e.slot_index;
    pa.prev_index = e.prev_index;
    pa.out_bytes = e.out_bytes;
    pa.dst_offset = e.chunk_off + ntiles;
    pa.flags = e.flags;
    pa.pool_high = e.pool_high;
    pa.total_bytes = e.total_bytes;
    PackArgs &ka = j.pack;
    ka.scratch = e.scratch;
    ka.chunk_words = g.max_chunk_words;
    ka.chunk_bits = e.chunk_bits;
    ka.nchunks = g.nchunks;
    ka.nsuper = g.nsuper;
    ka.table_bytes = g.table_bytes;
    ka.tile_prefix = tile;
    ka.dst = e.dst;
    ka.pool = e.pool;
    ka.dst_offset = e.chunk_off + ntiles;
    ka.flags = e.flags;
    j.wave0 = 0;
    j.tile0 = 0;
    return j;
}

static DecJob make_dec_job(const DecodeArgs &d)
{
    const CodecGeom g = codec_geom(d.f.ndim, d.f.n);
    DecJob j{};
    DecodeK &k = j.dec;
    k.f = d.f;
    k.dst = d.dst;
    k.stream = d.stream;
    k.pool = d.pool;
    k.slots = d.slots;
    k.slot_index = d.slot_index;
    k.nb0 = g.nb[0]; k.nb1 = g.nb[1]; k.nb2 = g.nb[2];
    k.nblocks = g.nblocks;
    k.nchunks = g.nchunks;
    k.kblk = g.kblk;
    k.nsuper = g.nsuper;
    k.table_bytes = g.table_bytes;
    k.flags = d.flags;
    k.vec = rows_vectorizable(d.f, d.dst);
    j.wave0 = 0;
    return j;
}

// ---- single-field kernels
// One wave per 64-chunk group; the _loop variants let a capped number of
// waves loop over the groups instead (same streams; a separate kernel,
// because the loop around the inlined body costs the one-pass kernel
// registers and speed).
template <int D>
__global__ __launch_bounds__(64) void encode_kernel(EncodeK k) { encode_body<D>(k, blockIdx.x); }

template <int D>
__global__ __launch_bounds__(64) void encode_loop_kernel(EncodeK k, long ngroups)
{
    for (long b = blockIdx.x; b < ngroups; b += gridDim.x) encode_body<D>(k, b);
}

__global__ __launch_bounds__(TILE) void tile_sum_kernel(const unsigned long long *chunk_bits, long nchunks,
                                                        unsigned long long *tile_sum)
{
    tile_sum_body(chunk_bits, nchunks, tile_sum, blockIdx.x);
}

__global__ __launch_bounds__(256) void plan_kernel(PlanArgs a) { plan_body(a); }

__global__ __launch_bounds__(TILE) void pack_kernel(PackArgs a) { pack_body(a, blockIdx.x); }

template <int D>
__global__ __launch_bounds__(64) void decode_kernel(DecodeK k) { decode_body<D>(k, blockIdx.x); }

template <int D>
__global__ __launch_bounds__(64) void decode_loop_kernel(DecodeK k, long ngroups)
{
    for (long b = blockIdx.x; b < ngroups; b += gridDim.x) decode_body<D>(k, b);
}

// ---- batched kernels: a block finds its field by binary search over the
// first block of every job
template <class J>
__device__ __forceinline__ int job_of(const J *__restrict__ jobs, int n, int blk, int J::*first)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].*first <= blk) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int D>
__global__ __launch_bounds__(64) void encode_batch_kernel(const EncJob *__restrict__ jobs, int n)
{
    const int j = job_of(jobs, n, blockIdx.x, &EncJob::wave0);
    encode_body<D>(jobs[j].enc, (long)blockIdx.x - jobs[j].wave0);
}

__global__ __launch_bounds__(TILE) void tile_sum_batch_kernel(const EncJob *__restrict__ jobs, int n)
{
    const int j = job_of(jobs, n, blockIdx.x, &EncJob::tile0);
    tile_sum_body(jobs[j].enc.chunk_bits, jobs[j].enc.nchunks, jobs[j].plan.tile_sum,
                  (long)blockIdx.x - jobs[j].tile0);
}

__global__ __launch_bounds__(256) void plan_batch_kernel(const EncJob *__restrict__ jobs)
{
    plan_body(jobs[blockIdx.x].plan);
}

__global__ __launch_bounds__(TILE) void pack_batch_kernel(const EncJob *__restrict__ jobs, int n)
{
    const int j = job_of(jobs, n, blockIdx.x, &EncJob::tile0);
    pack_body(jobs[j].pack, (long)blockIdx.x - jobs[j].tile0);
}

template <int D>
__global__ __launch_bounds__(64) void decode_batch_kernel(const DecJob *__restrict__ jobs, int n)
{
    const int j = job_of(jobs, n, blockIdx.x, &DecJob::wave0);
    decode_body<D>(jobs[j].dec, (long)blockIdx.x - jobs[j].wave0);
}

void codec_encode(const EncodeArgs &e, hipStream_t st)
{
    const EncJob j = make_enc_job(e);
    const long ngroups = j.enc.nchunks / 64;
    if (e.max_waves > 0 && e.max_waves < ngroups) {
        if (e.f.ndim == 3) hipLaunchKernelGGL(encode_loop_kernel<3>, dim3(e.max_waves), dim3(64), 0, st, j.enc, ngroups);
        else hipLaunchKernelGGL(encode_loop_kernel<2>, dim3(e.max_waves), dim3(64), 0, st, j.enc, ngroups);
    } else if (e.f.ndim == 3) {
        hipLaunchKernelGGL(encode_kernel<3>, dim3((unsigned)ngroups), dim3(64), 0, st, j.enc);
    } else {
        hipLaunchKernelGGL(encode_kernel<2>, dim3((unsigned)ngroups), dim3(64), 0, st, j.enc);
    }
    hipLaunchKernelGGL(tile_sum_kernel, dim3(j.plan.ntiles), dim3(TILE), 0, st, j.enc.chunk_bits,
                       j.enc.nchunks, j.plan.tile_sum);
    hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(256), 0, st, j.plan);
    hipLaunchKernelGGL(pack_kernel, dim3(j.plan.ntiles), dim3(TILE), 0, st, j.pack);
}

void codec_decode(const DecodeArgs &d, hipStream_t st)
{
    const DecJob j = make_dec_job(d);
    const long ngroups = j.dec.nchunks / 64;
    if (d.max_waves > 0 && d.max_waves < ngroups) {
        if (d.f.ndim == 3) hipLaunchKernelGGL(decode_loop_kernel<3>, dim3(d.max_waves), dim3(64), 0, st, j.dec, ngroups);
        else hipLaunchKernelGGL(decode_loop_kernel<2>, dim3(d.max_waves), dim3(64), 0, st, j.dec, ngroups);
    } else if (d.f.ndim == 3) {
        hipLaunchKernelGGL(decode_kernel<3>, dim3((unsigned)ngroups), dim3(64), 0, st, j.dec);
    } else {
        hipLaunchKernelGGL(decode_kernel<2>, dim3((unsigned)ngroups), dim3(64), 0, st, j.dec);
    }
}

size_t codec_job_bytes(bool encode) { return encode ? sizeof(EncJob) : sizeof(DecJob); }

int codec_resident_waves(int ndim, bool encode)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    hipError_t e;
    if (encode)
        e = ndim == 3 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, encode_loop_kernel<3>, 64, 0)
                      : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, encode_loop_kernel<2>, 64, 0);
    else
        e = ndim == 3 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, decode_loop_kernel<3>, 64, 0)
                      : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, decode_loop_kernel<2>, 64, 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return per_cu * cus;
}

void codec_encode_batch(const EncodeArgs *args, int n, void *host_jobs, void *dev_jobs, bool upload,
                        hipStream_t st)
{
    EncJob *h = (EncJob *)host_jobs;
    int waves = 0, tiles = 0;
    for (int i = 0; i < n; ++i) {
        h[i] = make_enc_job(args[i]);
        h[i].wave0 = waves;
        h[i].tile0 = tiles;
        waves += (int)(h[i].enc.nchunks / 64);
        tiles += h[i].plan.ntiles;
    }
    const EncJob *d = (const EncJob *)dev_jobs;
    if (upload) (void)hipMemcpyAsync(dev_jobs, host_jobs, (size_t)n * sizeof(EncJob), hipMemcpyHostToDevice, st);
    if (args[0].f.ndim == 3) hipLaunchKernelGGL(encode_batch_kernel<3>, dim3(waves), dim3(64), 0, st, d, n);
    else hipLaunchKernelGGL(encode_batch_kernel<2>, dim3(waves), dim3(64), 0, st, d, n);
    hipLaunchKernelGGL(tile_sum_batch_kernel, dim3(tiles), dim3(TILE), 0, st, d, n);
    hipLaunchKernelGGL(plan_batch_kernel, dim3(n), dim3(256), 0, st, d);
    hipLaunchKernelGGL(pack_batch_kernel, dim3(tiles), dim3(TILE), 0, st, d, n);
}

void codec_decode_batch(const DecodeArgs *args, int n, void *host_jobs, void *dev_jobs, bool upload,
                        hipStream_t st)
{
    DecJob *h = (DecJob *)host_jobs;
    int waves = 0;
    for (int i = 0; i < n; ++i) {
        h[i] = make_dec_job(args[i]);
        h[i].wave0 = waves;
        waves += (int)(h[i].dec.nchunks / 64);
    }
    const DecJob *d = (const DecJob *)dev_jobs;
    if (upload) (void)hipMemcpyAsync(dev_jobs, host_jobs, (size_t)n * sizeof(DecJob), hipMemcpyHostToDevice, st);
    if (args[0].f.ndim == 3) hipLaunchKernelGGL(decode_batch_kernel<3>, dim3(waves), dim3(64), 0, st, d, n);
    else hipLaunchKernelGGL(decode_batch_kernel<2>, dim3(waves), dim3(64), 0, st, d, n);
}

}  // namespace fwi
