// Leapfrog forward step and fused adjoint step + imaging condition for the
// acoustic wave equation (paper Eq. 1 and Eq. 4), gfx950.
//
// Both are one recurrence row solved for the new level, multiplied through
// by b = dt^2/m:
//   (1 + e) out = 2 c + b Lap_h c - (1 - e) u2 + b s,   e = kappa b sum d^2
// with c the middle level and u2 the oldest one (u^{k-1}, u^{k-2} forward;
// lam^{k+1}, lam^{k+2} adjoint).  The adjoint variant also accumulates
//   g -= u^k (out - 2 c + u2) / dt^2.
//
// Layout: every array a step touches (the levels, b, u^k, the gradient
// accumulator) shares one padded layout whose interior rows start on
// 128-byte L2 lines, and is addressed by 32-bit byte offsets from the
// allocation base (one scalar base + one vector offset per load).
//
// Work split: a workgroup owns a (y, z) tile and streams a chunk of x planes.
// Each lane keeps the 2R+1 x-neighbours of its column(s) in registers; the
// y and z neighbours of the current plane come from a double-buffered LDS
// tile whose centre is written from the register queue.  The loads of plane
// x+1 (queue value, halo ring, u2, b, and for the adjoint u^k and g) are
// issued before plane x is computed, and one barrier closes each plane.
// Lanes outside the grid compute nothing.  Extra workgroups at the end of a
// forward launch sample the receivers from the level the launch reads
// (u^{k-1}), so the first sweep needs no separate gather launch.
#include "internal.hpp"

namespace fwi {

namespace {

__device__ __forceinline__ int layer_depth(int i, int n, int nbl)
{
    int a = nbl - i;
    int b = i - (n - 1 - nbl);
    int d = a > b ? a : b;
    return d > 0 ? d : 0;
}

// load/store through a base pointer and an unsigned byte offset.  Every
// base is a device (global) array; the accesses say so, so that kernels
// whose pointers come from a table in memory (the batched ones) get global
// rather than flat instructions: a flat access also counts against the LDS
// wait counter, so every wait for an LDS read would wait for it as well.
typedef __attribute__((address_space(1))) float gfloat;

__device__ __forceinline__ float ld(const float *base, unsigned off)
{
    return *(const gfloat *)((const char *)base + off);
}

__device__ __forceinline__ float ldnt(const float *base, unsigned off)
{
    return __builtin_nontemporal_load((const gfloat *)((const char *)base + off));
}

__device__ __forceinline__ void st(float *base, unsigned off, float v)
{
    *(gfloat *)((char *)base + off) = v;
}

// streaming store: the 3D levels and gradient are far larger than the
// caches and are next read a whole step later
__device__ __forceinline__ void stnt(float *base, unsigned off, float v)
{
    __builtin_nontemporal_store(v, (gfloat *)((char *)base + off));
}

// Increment out - c of the new level.  The recurrence row is written around
// the current level,
//   (1 + e) (out - c) = (1 - e) (c - u2) + b (Lap_h c + s),
// so the small time difference c - u2 is formed before anything is rounded
// (FP32 rounding of 2c - u2 is what drifts over thousands of steps).
template <bool ADJ>
__device__ __forceinline__ float increment(const StepParams &p, int dsum, bool is_src, float c, float lap,
                                           float u2v, float bb)
{
    const float d = c - u2v;
    float rhs = lap;
    if (!ADJ && is_src) rhs += p.wav[p.step];
    if (dsum == 0) return fmaf(bb, rhs, d);
    const float e = p.kappa * bb * (float)dsum;
    return fmaf(bb, rhs, (1.0f - e) * d) / (1.0f + e);
}

// one axis pair of the Laplacian without the centre weight:
// a_0 = -2 sum_k a_k, so Lap_h c = sum_k w_k sum_axes (u_-k + u_+k - 2c), and
// each pair minus 2c is small where the field is smooth (no large centre
// term left to cancel)
__device__ __forceinline__ float pair2(float a, float b, float c)
{
    return fmaf(-2.0f, c, a + b);
}

__device__ __forceinline__ void gather_block(const StepParams &p, int blk)
{
    const int j = blk * (int)(blockDim.x * blockDim.y) + (int)(threadIdx.y * blockDim.x + threadIdx.x);
    if (j < p.nrec) p.grow[j] = ld(p.u1, 4u * (unsigned)p.rec_off[j]);
}

// ------------------------------------------------------------------- 3D
// Workgroup = 64 (z) x 8 (y) lanes; each lane owns RPL rows (ty + 8 j) of a
// 64 x 8 RPL (z, y) tile.  Tiles are numbered z fastest, then y, then x
// chunk.  Workgroups are dealt to the 8 XCDs round robin; `remap` 1 hands
// out tiles so that each XCD works on one contiguous range, `remap` 2 so
// that the z tiles of one (y, x chunk) column go to one XCD in a row (their
// z halos are then read from that XCD's L2) while columns still go round
// robin; `remap` 3 and 4 hand each XCD groups of G = 2 or 4 consecutive
// columns (y neighbours of one x chunk) in a row, so that the y halos inside
// a group are read from that XCD's L2 too.  Read-once streams (u2, b, u^k,
// g) use non-temporal loads.
__device__ __forceinline__ void tile_coords(int hw, int nwg, int ntz, int nty, int remap, int &tzi,
                                            int &tyi, int &txi, bool &valid)
{
    int logical = hw;
    if (remap == 1) {
        const int per = (nwg + 7) >> 3;
        logical = (hw & 7) * per + (hw >> 3);
    } else if (remap >= 2) {
        // a bijection of [0, launched) when launched is a multiple of
        // 8 G ntz: the XCD's k-th workgroup takes z tile k % ntz of its
        // (k / ntz)-th column, columns in groups of G per XCD
        const int lg = remap - 2;
        const int k = hw >> 3, cx = k / ntz;
        const int col = ((((cx >> lg) << 3) + (hw & 7)) << lg) + (cx & ((1 << lg) - 1));
        logical = col * ntz + k % ntz;
    }
    valid = logical < nwg;
    tzi = logical % ntz;
    const int rest = logical / ntz;
    tyi = rest % nty;
    txi = rest / nty;
}

template <int R, bool ADJ, int RPL>
__device__ __forceinline__ void step3d_body(const StepParams &p, int hw, int ntz, int nty, int nwg,
                                            int launched)
{
    constexpr int ROWS = 8 * RPL;
    __shared__ float tile[2][ROWS + 2 * R][TILE_Z + 2 * R];
    if (hw >= launched) {                          // receiver sampling blocks
        gather_block(p, hw - launched);
        return;
    }
    int tzi, tyi, txi;
    bool valid;
    tile_coords(hw, nwg, ntz, nty, p.remap, tzi, tyi, txi, valid);
    if (!valid) return;                            // whole workgroup, before any barrier

    const int tz = threadIdx.x;
    const int ty = threadIdx.y;
    const int z0 = tzi * TILE_Z;
    const int y0 = tyi * ROWS;
    const int z = z0 + tz;
    const int xb = txi * p.xchunk;
    const int xe = min(xb + p.xchunk, p.nx);
    const bool zin = z < p.nz;
    // byte strides and offsets (unsigned arithmetic; every result is in range)
    const unsigned bsx = 4u * (unsigned)p.psx, bsy = 4u * (unsigned)p.psy;
    const unsigned org = 4u * (unsigned)p.origin;
    const unsigned srcb = p.src >= 0 ? org + 4u * (unsigned)p.src : 0xFFFFFFFFu;
    const float *__restrict__ u1 = p.u1;
    const float *__restrict__ u2 = p.u2;
    const float *__restrict__ bq = p.b;
    const bool hy = ty < R;
    const unsigned hy_top = org + (unsigned)(y0 - R + ty) * bsy + 4u * z;
    const unsigned hy_bot = org + (unsigned)(y0 + ROWS + ty) * bsy + 4u * z;
    const bool hzl = tz < R, hzr = tz >= TILE_Z - R;
    const bool hz = hzl || hzr;
    const unsigned hz_off = 4u * (unsigned)(hzl ? (z0 - R + tz) : (z + R));
    const int hcol = hzl ? tz : tz + 2 * R;
    const unsigned col0 = org + (unsigned)(y0 + ty) * bsy + 4u * z;   // row j at + 8 j bsy
    const unsigned hz0 = org + (unsigned)(y0 + ty) * bsy + hz_off;
    const unsigned rstep = 8u * bsy;
    const int dz = layer_depth(z, p.nz, p.nbl);
    bool act[RPL];
    int dyz[RPL];
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
        const int y = y0 + ty + 8 * j;
        act[j] = zin && y < p.ny;
        const int dy = layer_depth(y, p.ny, p.nbl);
        dyz[j] = dy * dy + dz * dz;
    }

    float q[RPL][2 * R + 1];
#pragma unroll
    for (int j = 0; j < RPL; ++j)
#pragma unroll
        for (int i = 0; i <= 2 * R; ++i) q[j][i] = ld(u1, col0 + j * rstep + (unsigned)(xb - R + i) * bsx);
    {
        const unsigned pl = (unsigned)xb * bsx;
#pragma unroll
        for (int j = 0; j < RPL; ++j) tile[0][ty + 8 * j + R][tz + R] = q[j][R];
        if (hy) {
            tile[0][ty][tz + R] = ld(u1, pl + hy_top);
            tile[0][ty + ROWS + R][tz + R] = ld(u1, pl + hy_bot);
        }
        if (hz) {
#pragma unroll
            for (int j = 0; j < RPL; ++j) tile[0][ty + 8 * j + R][hcol] = ld(u1, pl + hz0 + j * rstep);
        }
    }
    unsigned pa = col0 + (unsigned)xb * bsx;            // row j at + j rstep
    float u2v[RPL], bv[RPL], ukv[RPL], gv[RPL];
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
        const unsigned o = pa + j * rstep;
        u2v[j] = act[j] ? ldnt(u2, o) : 0.f;
        bv[j] = act[j] ? ldnt(bq, o) : 0.f;
        ukv[j] = (ADJ && act[j]) ? ldnt(p.uk, o) : 0.f;
        gv[j] = (ADJ && act[j]) ? ldnt(p.g, o) : 0.f;
    }
    __syncthreads();

    for (int x = xb; x < xe; ++x) {
        const int cur = (x - xb) & 1;
        const bool nxt = x + 1 < xe;
        // ---- issue the loads of plane x+1 (halo first: needed soonest)
        float nq[RPL], nhz[RPL], nu2[RPL], nb_[RPL], nuk[RPL], ng[RPL];
        float nht = 0.f, nhb = 0.f;
#pragma unroll
        for (int j = 0; j < RPL; ++j) nq[j] = nhz[j] = nu2[j] = nb_[j] = nuk[j] = ng[j] = 0.f;
        if (nxt) {
            const unsigned pl = (unsigned)(x + 1) * bsx;
            if (hy) {
                nht = ld(u1, pl + hy_top);
                nhb = ld(u1, pl + hy_bot);
            }
            if (hz) {
#pragma unroll
                for (int j = 0; j < RPL; ++j) nhz[j] = ld(u1, pl + hz0 + j * rstep);
            }
#pragma unroll
            for (int j = 0; j < RPL; ++j) nq[j] = ld(u1, col0 + j * rstep + pl + (unsigned)R * bsx);
#pragma unroll
            for (int j = 0; j < RPL; ++j) {
                const unsigned na = pa + bsx + j * rstep;
                if (act[j]) {
                    nu2[j] = ldnt(u2, na);
                    nb_[j] = ldnt(bq, na);
                    if (ADJ) { nuk[j] = ldnt(p.uk, na); ng[j] = ldnt(p.g, na); }
                }
            }
        }
        // ---- plane x
        const int dx = layer_depth(x, p.nx, p.nbl);
#pragma unroll
        for (int j = 0; j < RPL; ++j) {
            if (!act[j]) continue;
            const int r = ty + 8 * j + R;
            const float c = q[j][R];
            float lap = 0.0f;
#pragma unroll
            for (int k = 1; k <= R; ++k)
                lap = fmaf(p.w[k], pair2(q[j][R - k], q[j][R + k], c) +
                                   pair2(tile[cur][r - k][tz + R], tile[cur][r + k][tz + R], c) +
                                   pair2(tile[cur][r][tz + R - k], tile[cur][r][tz + R + k], c), lap);
            const unsigned o = pa + j * rstep;
            const float inc = increment<ADJ>(p, dx * dx + dyz[j], o == srcb, c, lap, u2v[j], bv[j]);
            stnt(p.out, o, c + inc);
            // imaging: out - 2c + u2 = (out - c) - (c - u2)
            if (ADJ) stnt(p.g, o, gv[j] - ukv[j] * (inc - (c - u2v[j])) * p.inv_dt2);
        }
        if (!nxt) break;
        // ---- advance the queues and stage plane x+1 in the other buffer
        const int nb = cur ^ 1;
#pragma unroll
        for (int j = 0; j < RPL; ++j) {
#pragma unroll
            for (int i = 0; i < 2 * R; ++i) q[j][i] = q[j][i + 1];
            q[j][2 * R] = nq[j];
            tile[nb][ty + 8 * j + R][tz + R] = q[j][R];
            if (hz) tile[nb][ty + 8 * j + R][hcol] = nhz[j];
            u2v[j] = nu2[j];
            bv[j] = nb_[j];
            if (ADJ) { ukv[j] = nuk[j]; gv[j] = ng[j]; }
        }
        if (hy) {
            tile[nb][ty][tz + R] = nht;
            tile[nb][ty + ROWS + R][tz + R] = nhb;
        }
        pa += bsx;
        __syncthreads();
    }
}

// Same step with the loads of plane x+2 issued while plane x is computed
// (two planes in flight per workgroup instead of one).
template <int R, bool ADJ, int RPL>
__device__ __forceinline__ void step3d_body_deep(const StepParams &p, int hw, int ntz, int nty, int nwg,
                                            int launched)
{
    constexpr int ROWS = 8 * RPL;
    __shared__ float tile[2][ROWS + 2 * R][TILE_Z + 2 * R];
    if (hw >= launched) {                          // receiver sampling blocks
        gather_block(p, hw - launched);
        return;
    }
    int tzi, tyi, txi;
    bool valid;
    tile_coords(hw, nwg, ntz, nty, p.remap, tzi, tyi, txi, valid);
    if (!valid) return;                            // whole workgroup, before any barrier

    const int tz = threadIdx.x;
    const int ty = threadIdx.y;
    const int z0 = tzi * TILE_Z;
    const int y0 = tyi * ROWS;
    const int z = z0 + tz;
    const int xb = txi * p.xchunk;
    const int xe = min(xb + p.xchunk, p.nx);
    const bool zin = z < p.nz;
    // byte strides and offsets (unsigned arithmetic; every result is in range)
    const unsigned bsx = 4u * (unsigned)p.psx, bsy = 4u * (unsigned)p.psy;
    const unsigned org = 4u * (unsigned)p.origin;
    const unsigned srcb = p.src >= 0 ? org + 4u * (unsigned)p.src : 0xFFFFFFFFu;
    const float *__restrict__ u1 = p.u1;
    const float *__restrict__ u2 = p.u2;
    const float *__restrict__ bq = p.b;
    const bool hy = ty < R;
    const unsigned hy_top = org + (unsigned)(y0 - R + ty) * bsy + 4u * z;
    const unsigned hy_bot = org + (unsigned)(y0 + ROWS + ty) * bsy + 4u * z;
    const bool hzl = tz < R, hzr = tz >= TILE_Z - R;
    const bool hz = hzl || hzr;
    const unsigned hz_off = 4u * (unsigned)(hzl ? (z0 - R + tz) : (z + R));
    const int hcol = hzl ? tz : tz + 2 * R;
    const unsigned col0 = org + (unsigned)(y0 + ty) * bsy + 4u * z;   // row j at + 8 j bsy
    const unsigned hz0 = org + (unsigned)(y0 + ty) * bsy + hz_off;
    const unsigned rstep = 8u * bsy;
    const int dz = layer_depth(z, p.nz, p.nbl);
    bool act[RPL];
    int dyz[RPL];
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
        const int y = y0 + ty + 8 * j;
        act[j] = zin && y < p.ny;
        const int dy = layer_depth(y, p.ny, p.nbl);
        dyz[j] = dy * dy + dz * dz;
    }

    float q[RPL][2 * R + 1];
#pragma unroll
    for (int j = 0; j < RPL; ++j)
#pragma unroll
        for (int i = 0; i <= 2 * R; ++i) q[j][i] = ld(u1, col0 + j * rstep + (unsigned)(xb - R + i) * bsx);
    {
        const unsigned pl = (unsigned)xb * bsx;
#pragma unroll
        for (int j = 0; j < RPL; ++j) tile[0][ty + 8 * j + R][tz + R] = q[j][R];
        if (hy) {
            tile[0][ty][tz + R] = ld(u1, pl + hy_top);
            tile[0][ty + ROWS + R][tz + R] = ld(u1, pl + hy_bot);
        }
        if (hz) {
#pragma unroll
            for (int j = 0; j < RPL; ++j) tile[0][ty + 8 * j + R][hcol] = ld(u1, pl + hz0 + j * rstep);
        }
    }
    unsigned pa = col0 + (unsigned)xb * bsx;            // row j at + j rstep
    float u2v[RPL], bv[RPL], ukv[RPL], gv[RPL];
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
        const unsigned o = pa + j * rstep;
        u2v[j] = act[j] ? ldnt(u2, o) : 0.f;
        bv[j] = act[j] ? ldnt(bq, o) : 0.f;
        ukv[j] = (ADJ && act[j]) ? ldnt(p.uk, o) : 0.f;
        gv[j] = (ADJ && act[j]) ? ldnt(p.g, o) : 0.f;
    }
    // loads of one future plane: queue value (R planes further), halo ring, u2, b (u^k, g)
    struct Ld {
        float q[RPL], hz[RPL], u2[RPL], b[RPL], uk[RPL], g[RPL];
        float ht, hb;
    };
    auto issue = [&](Ld &L, int xp) {
        const unsigned pl = (unsigned)xp * bsx;
        L.ht = L.hb = 0.f;
#pragma unroll
        for (int j = 0; j < RPL; ++j) L.q[j] = L.hz[j] = L.u2[j] = L.b[j] = L.uk[j] = L.g[j] = 0.f;
        if (hy) {
            L.ht = ld(u1, pl + hy_top);
            L.hb = ld(u1, pl + hy_bot);
        }
        if (hz) {
#pragma unroll
            for (int j = 0; j < RPL; ++j) L.hz[j] = ld(u1, pl + hz0 + j * rstep);
        }
#pragma unroll
        for (int j = 0; j < RPL; ++j) L.q[j] = ld(u1, col0 + j * rstep + pl + (unsigned)R * bsx);
        const unsigned na0 = col0 + pl;
#pragma unroll
        for (int j = 0; j < RPL; ++j) {
            const unsigned na = na0 + j * rstep;
            if (act[j]) {
                L.u2[j] = ldnt(u2, na);
                L.b[j] = ldnt(bq, na);
                if (ADJ) { L.uk[j] = ldnt(p.uk, na); L.g[j] = ldnt(p.g, na); }
            }
        }
    };
    Ld A, B;
    if (xb + 1 < xe) issue(A, xb + 1);
    __syncthreads();

    for (int x = xb; x < xe; ++x) {
        const int cur = (x - xb) & 1;
        if (x + 2 < xe) issue(B, x + 2);
        // ---- plane x
        const int dx = layer_depth(x, p.nx, p.nbl);
#pragma unroll
        for (int j = 0; j < RPL; ++j) {
            if (!act[j]) continue;
            const int r = ty + 8 * j + R;
            const float c = q[j][R];
            float lap = 0.0f;
#pragma unroll
            for (int k = 1; k <= R; ++k)
                lap = fmaf(p.w[k], pair2(q[j][R - k], q[j][R + k], c) +
                                   pair2(tile[cur][r - k][tz + R], tile[cur][r + k][tz + R], c) +
                                   pair2(tile[cur][r][tz + R - k], tile[cur][r][tz + R + k], c), lap);
            const unsigned o = pa + j * rstep;
            const float inc = increment<ADJ>(p, dx * dx + dyz[j], o == srcb, c, lap, u2v[j], bv[j]);
            stnt(p.out, o, c + inc);
            // imaging: out - 2c + u2 = (out - c) - (c - u2)
            if (ADJ) stnt(p.g, o, gv[j] - ukv[j] * (inc - (c - u2v[j])) * p.inv_dt2);
        }
        if (x + 1 >= xe) break;
        // ---- advance the queues and stage plane x+1 (loads issued one plane ago)
        const int nb = cur ^ 1;
#pragma unroll
        for (int j = 0; j < RPL; ++j) {
#pragma unroll
            for (int i = 0; i < 2 * R; ++i) q[j][i] = q[j][i + 1];
            q[j][2 * R] = A.q[j];
            tile[nb][ty + 8 * j + R][tz + R] = q[j][R];
            if (hz) tile[nb][ty + 8 * j + R][hcol] = A.hz[j];
            u2v[j] = A.u2[j];
            bv[j] = A.b[j];
            if (ADJ) { ukv[j] = A.uk[j]; gv[j] = A.g[j]; }
        }
        if (hy) {
            tile[nb][ty][tz + R] = A.ht;
            tile[nb][ty + ROWS + R][tz + R] = A.hb;
        }
        A = B;
        pa += bsx;
        __syncthreads();
    }
}

template <int R, bool ADJ, int RPL>
__global__ __launch_bounds__(TILE_Z * 8)
void step3d_kernel(StepParams p, int ntz, int nty, int nwg, int launched)
{
    step3d_body<R, ADJ, RPL>(p, blockIdx.x, ntz, nty, nwg, launched);
}

template <int R, bool ADJ>
__global__ __launch_bounds__(TILE_Z * 8)
void step3d_deep_kernel(StepParams p, int ntz, int nty, int nwg, int launched)
{
    step3d_body_deep<R, ADJ, 2>(p, blockIdx.x, ntz, nty, nwg, launched);
}

// ----------------------------------------------------- 3D, 8-byte lanes
// Same streaming scheme with two consecutive z points per lane: a wave
// covers 128 z points, every global access moves 8 bytes per lane and the
// z neighbours come from 8-byte LDS reads.  The tile is 128 (z) x 8 RPL (y);
// wider z tiles halve the z-halo lines per point and the wider accesses keep
// more bytes in flight per load instruction.  Lanes whose second point lies
// past the field end load padding (zero) and store only the first point.
typedef float f2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ f2v ld2(const float *base, unsigned off)
{
    return *(const f2v *)((const char *)base + off);
}

__device__ __forceinline__ f2v ldnt2(const float *base, unsigned off)
{
    return __builtin_nontemporal_load((const f2v *)((const char *)base + off));
}

__device__ __forceinline__ void st2(float *base, unsigned off, f2v v, bool both)
{
    if (both) __builtin_nontemporal_store(v, (f2v *)((char *)base + off));
    else __builtin_nontemporal_store(v.x, (float *)((char *)base + off));
}

template <int R, bool ADJ, int RPL>
__device__ __forceinline__ void step3w_body(const StepParams &p, int hw, int ntz, int nty, int nwg,
                                            int launched)
{
    constexpr int ROWS = 8 * RPL;
    constexpr int TZ = TILE_ZW;
    constexpr int WL = TZ + 2 * R;                 // LDS row (floats)
    constexpr int HP = R / 2;                      // z-halo pairs per side
    __shared__ __attribute__((aligned(16))) float tile[2][ROWS + 2 * R][WL];
    if (hw >= launched) {                          // receiver sampling blocks
        gather_block(p, hw - launched);
        return;
    }
    int tzi, tyi, txi;
    bool valid;
    tile_coords(hw, nwg, ntz, nty, p.remap, tzi, tyi, txi, valid);
    if (!valid) return;                            // whole workgroup, before any barrier

    const int tz = threadIdx.x;
    const int ty = threadIdx.y;
    const int z0 = tzi * TZ;
    const int y0 = tyi * ROWS;
    const int za = z0 + 2 * tz;                    // the lane's points za, za + 1
    const int xb = txi * p.xchunk;
    const int xe = min(xb + p.xchunk, p.nx);
    const bool zin = za < p.nz;
    const bool both = za + 1 < p.nz;
    const unsigned bsx = 4u * (unsigned)p.psx, bsy = 4u * (unsigned)p.psy;
    const unsigned org = 4u * (unsigned)p.origin;
    const unsigned srcb = p.src >= 0 ? org + 4u * (unsigned)p.src : 0xFFFFFFFFu;
    const float *__restrict__ u1 = p.u1;
    const float *__restrict__ u2 = p.u2;
    const float *__restrict__ bq = p.b;
    const bool hy = ty < R;
    const unsigned hy_top = org + (unsigned)(y0 - R + ty) * bsy + 4u * za;
    const unsigned hy_bot = org + (unsigned)(y0 + ROWS + ty) * bsy + 4u * za;
    // z halo: lanes 0..HP-1 load the pairs left of the tile, lanes
    // 64-HP..63 the pairs right of it
    const bool hzl = tz < HP, hzr = tz >= 64 - HP;
    const bool hz = hzl || hzr;
    const int hzz = hzl ? z0 - R + 2 * tz : z0 + TZ + 2 * (tz - (64 - HP));
    const int hcol = hzl ? 2 * tz : TZ + R + 2 * (tz - (64 - HP));
    const int ccol = R + 2 * tz;                   // LDS column of za
    const unsigned col0 = org + (unsigned)(y0 + ty) * bsy + 4u * za;
    const unsigned hz0 = org + (unsigned)(y0 + ty) * bsy + 4u * (unsigned)hzz;
    const unsigned rstep = 8u * bsy;
    const int dza = layer_depth(za, p.nz, p.nbl), dzb = layer_depth(za + 1, p.nz, p.nbl);
    bool act[RPL];
    int dya[RPL];
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
        const int y = y0 + ty + 8 * j;
        act[j] = zin && y < p.ny;
        dya[j] = layer_depth(y, p.ny, p.nbl);
        dya[j] *= dya[j];
    }

    f2v q[RPL][2 * R + 1];
#pragma unroll
    for (int j = 0; j < RPL; ++j)
#pragma unroll
        for (int i = 0; i <= 2 * R; ++i) q[j][i] = ld2(u1, col0 + j * rstep + (unsigned)(xb - R + i) * bsx);
    {
        const unsigned pl = (unsigned)xb * bsx;
#pragma unroll
        for (int j = 0; j < RPL; ++j) *(f2v *)&tile[0][ty + 8 * j + R][ccol] = q[j][R];
        if (hy) {
            *(f2v *)&tile[0][ty][ccol] = ld2(u1, pl + hy_top);
            *(f2v *)&tile[0][ty + ROWS + R][ccol] = ld2(u1, pl + hy_bot);
        }
        if (hz) {
#pragma unroll
            for (int j = 0; j < RPL; ++j) *(f2v *)&tile[0][ty + 8 * j + R][hcol] = ld2(u1, pl + hz0 + j * rstep);
        }
    }
    unsigned pa = col0 + (unsigned)xb * bsx;
    const f2v zero2 = {0.f, 0.f};
    f2v u2v[RPL], bv[RPL], ukv[RPL], gv[RPL];
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
        const unsigned o = pa + j * rstep;
        u2v[j] = act[j] ? ldnt2(u2, o) : zero2;
        bv[j] = act[j] ? ldnt2(bq, o) : zero2;
        ukv[j] = (ADJ && act[j]) ? ldnt2(p.uk, o) : zero2;
        gv[j] = (ADJ && act[j]) ? ldnt2(p.g, o) : zero2;
    }
    __syncthreads();

    for (int x = xb; x < xe; ++x) {
        const int cur = (x - xb) & 1;
        const bool nxt = x + 1 < xe;
        f2v nq[RPL], nhz[RPL], nu2[RPL], nb_[RPL], nuk[RPL], ng[RPL];
        f2v nht = zero2, nhb = zero2;
#pragma unroll
        for (int j = 0; j < RPL; ++j) nq[j] = nhz[j] = nu2[j] = nb_[j] = nuk[j] = ng[j] = zero2;
        if (nxt) {
            const unsigned pl = (unsigned)(x + 1) * bsx;
            if (hy) {
                nht = ld2(u1, pl + hy_top);
                nhb = ld2(u1, pl + hy_bot);
            }
            if (hz) {
#pragma unroll
                for (int j = 0; j < RPL; ++j) nhz[j] = ld2(u1, pl + hz0 + j * rstep);
            }
#pragma unroll
            for (int j = 0; j < RPL; ++j) nq[j] = ld2(u1, col0 + j * rstep + pl + (unsigned)R * bsx);
#pragma unroll
            for (int j = 0; j < RPL; ++j) {
                const unsigned na = pa + bsx + j * rstep;
                if (act[j]) {
                    nu2[j] = ldnt2(u2, na);
                    nb_[j] = ldnt2(bq, na);
                    if (ADJ) { nuk[j] = ldnt2(p.uk, na); ng[j] = ldnt2(p.g, na); }
                }
            }
        }
        const int dx = layer_depth(x, p.nx, p.nbl);
#pragma unroll
        for (int j = 0; j < RPL; ++j) {
            if (!act[j]) continue;
            const int r = ty + 8 * j + R;
            const f2v c = q[j][R];
            // zr[i] = tile row r at column ccol - R + i, i = 0..2R+1
            float zr[2 * R + 2];
#pragma unroll
            for (int m = 0; m <= R; ++m) {
                const f2v v = m == HP ? c : *(const f2v *)&tile[cur][r][ccol - R + 2 * m];
                zr[2 * m] = v.x;
                zr[2 * m + 1] = v.y;
            }
            float la = 0.0f, lb = 0.0f;
#pragma unroll
            for (int k = 1; k <= R; ++k) {
                const f2v ym = *(const f2v *)&tile[cur][r - k][ccol];
                const f2v yp = *(const f2v *)&tile[cur][r + k][ccol];
                la = fmaf(p.w[k], pair2(q[j][R - k].x, q[j][R + k].x, c.x) + pair2(ym.x, yp.x, c.x) +
                                  pair2(zr[R - k], zr[R + k], c.x), la);
                lb = fmaf(p.w[k], pair2(q[j][R - k].y, q[j][R + k].y, c.y) + pair2(ym.y, yp.y, c.y) +
                                  pair2(zr[R + 1 - k], zr[R + 1 + k], c.y), lb);
            }
            const unsigned o = pa + j * rstep;
            const int dxy = dx * dx + dya[j];
            f2v inc, ov;
            inc.x = increment<ADJ>(p, dxy + dza * dza, o == srcb, c.x, la, u2v[j].x, bv[j].x);
            inc.y = increment<ADJ>(p, dxy + dzb * dzb, o + 4u == srcb, c.y, lb, u2v[j].y, bv[j].y);
            ov.x = c.x + inc.x;
            ov.y = c.y + inc.y;
            st2(p.out, o, ov, both);
            if (ADJ) {
                f2v gn;
                gn.x = gv[j].x - ukv[j].x * (inc.x - (c.x - u2v[j].x)) * p.inv_dt2;
                gn.y = gv[j].y - ukv[j].y * (inc.y - (c.y - u2v[j].y)) * p.inv_dt2;
                st2(p.g, o, gn, both);
            }
        }
        if (!nxt) break;
        const int nb = cur ^ 1;
#pragma unroll
        for (int j = 0; j < RPL; ++j) {
#pragma unroll
            for (int i = 0; i < 2 * R; ++i) q[j][i] = q[j][i + 1];
            q[j][2 * R] = nq[j];
            *(f2v *)&tile[nb][ty + 8 * j + R][ccol] = q[j][R];
            if (hz) *(f2v *)&tile[nb][ty + 8 * j + R][hcol] = nhz[j];
            u2v[j] = nu2[j];
            bv[j] = nb_[j];
            if (ADJ) { ukv[j] = nuk[j]; gv[j] = ng[j]; }
        }
        if (hy) {
            *(f2v *)&tile[nb][ty][ccol] = nht;
            *(f2v *)&tile[nb][ty + ROWS + R][ccol] = nhb;
        }
        pa += bsx;
        __syncthreads();
    }
}

template <int R, bool ADJ, int RPL>
__global__ __launch_bounds__(64 * 8)
void step3w_kernel(StepParams p, int ntz, int nty, int nwg, int launched)
{
    step3w_body<R, ADJ, RPL>(p, blockIdx.x, ntz, nty, nwg, launched);
}

// ------------------------------------------------------------------- 2D
// Workgroup = 256 lanes along z, one row each, streaming x two planes per
// step of the loop: the z neighbours of both planes come from LDS rows
// written together, so one barrier serves two planes; the x neighbours sit
// in a register queue (planes x - R .. x + R + 1).
template <int R, bool ADJ>
__device__ __forceinline__ void step2d_body(const StepParams &p, int hw, int ntz, int nwg)
{
    __shared__ float row[2][2][TILE_Z2 + 2 * R];
    if (hw >= nwg) {
        gather_block(p, hw - nwg);
        return;
    }
    const int tzi = hw % ntz;
    const int txi = hw / ntz;
    const int tz = threadIdx.x;
    const int z0 = tzi * TILE_Z2;
    const int z = z0 + tz;
    const int xb = txi * p.xchunk;
    const int xe = min(xb + p.xchunk, p.nx);
    const bool act = z < p.nz;
    const unsigned bsx = 4u * (unsigned)p.psx, org = 4u * (unsigned)p.origin;
    const unsigned srcb = p.src >= 0 ? org + 4u * (unsigned)p.src : 0xFFFFFFFFu;
    const float *__restrict__ u1 = p.u1;
    const bool hzl = tz < R, hzr = tz >= TILE_Z2 - R;
    const bool halo = hzl || hzr;
    const int hslot = hzl ? tz : tz + 2 * R;
    const unsigned hz_off = org + 4u * (unsigned)(hzl ? (z0 - R + tz) : (z + R));
    const unsigned col = org + 4u * z;
    const int dz = layer_depth(z, p.nz, p.nbl);

    // q[i]: u1 on plane x - R + i (x the first plane of the pair); u2, b,
    // (uk, g) of planes x and x + 1 in [0] and [1]
    float q[2 * R + 2];
    float u2v[2], bb[2], ukv[2], gv[2];
    const bool two = xb + 1 < xe;
#pragma unroll
    for (int i = 0; i <= 2 * R; ++i) q[i] = ld(u1, col + (unsigned)(xb - R + i) * bsx);
    q[2 * R + 1] = two ? ld(u1, col + (unsigned)(xb + R + 1) * bsx) : 0.f;
    unsigned pa = col + (unsigned)xb * bsx;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const bool in = j == 0 || two;
        u2v[j] = in && act ? ldnt(p.u2, pa + (unsigned)j * bsx) : 0.f;
        bb[j] = in && act ? ldnt(p.b, pa + (unsigned)j * bsx) : 0.f;
        ukv[j] = ADJ && in && act ? ldnt(p.uk, pa + (unsigned)j * bsx) : 0.f;
        gv[j] = ADJ && in && act ? ldnt(p.g, pa + (unsigned)j * bsx) : 0.f;
    }
    row[0][0][tz + R] = q[R];
    row[0][1][tz + R] = q[R + 1];
    if (halo) {
        row[0][0][hslot] = ld(u1, (unsigned)xb * bsx + hz_off);
        row[0][1][hslot] = two ? ld(u1, (unsigned)(xb + 1) * bsx + hz_off) : 0.f;
    }
    __syncthreads();
    for (int x = xb; x < xe; x += 2) {
        const int cur = ((x - xb) >> 1) & 1;
        // planes of the next pair that exist in the chunk
        const bool n0 = x + 2 < xe, n1 = x + 3 < xe;
        float nq0 = 0.f, nq1 = 0.f, nh0 = 0.f, nh1 = 0.f;
        float nu2[2] = {0.f, 0.f}, nbv[2] = {0.f, 0.f}, nuk[2] = {0.f, 0.f}, ng[2] = {0.f, 0.f};
        if (n0) {
            if (halo) nh0 = ld(u1, (unsigned)(x + 2) * bsx + hz_off);
            nq0 = ld(u1, col + (unsigned)(x + 2 + R) * bsx);
            if (act) {
                nu2[0] = ldnt(p.u2, pa + 2 * bsx);
                nbv[0] = ldnt(p.b, pa + 2 * bsx);
                if (ADJ) { nuk[0] = ldnt(p.uk, pa + 2 * bsx); ng[0] = ldnt(p.g, pa + 2 * bsx); }
            }
        }
        if (n1) {
            if (halo) nh1 = ld(u1, (unsigned)(x + 3) * bsx + hz_off);
            nq1 = ld(u1, col + (unsigned)(x + 3 + R) * bsx);
            if (act) {
                nu2[1] = ldnt(p.u2, pa + 3 * bsx);
                nbv[1] = ldnt(p.b, pa + 3 * bsx);
                if (ADJ) { nuk[1] = ldnt(p.uk, pa + 3 * bsx); ng[1] = ldnt(p.g, pa + 3 * bsx); }
            }
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            if (j == 1 && x + 1 >= xe) break;
            if (act) {
                const float c = q[R + j];
                float lap = 0.0f;
#pragma unroll
                for (int k = 1; k <= R; ++k)
                    lap = fmaf(p.w[k], pair2(q[R + j - k], q[R + j + k], c) +
                                       pair2(row[cur][j][tz + R - k], row[cur][j][tz + R + k], c), lap);
                const int dx = layer_depth(x + j, p.nx, p.nbl);
                const unsigned pj = pa + (unsigned)j * bsx;
                const float inc = increment<ADJ>(p, dx * dx + dz * dz, pj == srcb, c, lap, u2v[j], bb[j]);
                st(p.out, pj, c + inc);
                if (ADJ) st(p.g, pj, gv[j] - ukv[j] * (inc - (c - u2v[j])) * p.inv_dt2);
            }
        }
        if (!n0) break;
#pragma unroll
        for (int i = 0; i < 2 * R; ++i) q[i] = q[i + 2];
        q[2 * R] = nq0;
        q[2 * R + 1] = nq1;
        row[cur ^ 1][0][tz + R] = q[R];
        row[cur ^ 1][1][tz + R] = q[R + 1];
        if (halo) {
            row[cur ^ 1][0][hslot] = nh0;
            row[cur ^ 1][1][hslot] = nh1;
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            u2v[j] = nu2[j]; bb[j] = nbv[j];
            if (ADJ) { ukv[j] = nuk[j]; gv[j] = ng[j]; }
        }
        pa += 2 * bsx;
        __syncthreads();
    }
}

template <int R, bool ADJ>
__global__ __launch_bounds__(TILE_Z2)
void step2d_kernel(StepParams p, int ntz, int nwg)
{
    step2d_body<R, ADJ>(p, blockIdx.x, ntz, nwg);
}

// ---------------------------------------------------------------- batched
// One launch covers several shots: entry s owns workgroups
// [first_s, first_{s+1}); a workgroup finds its entry by binary search (over
// the kernel-argument copy of `first` when the batch has at most
// BATCH_INDEX shots, else over the table) and runs the same body as the
// single-shot kernel on that entry's parameters.
constexpr int BATCH_INDEX = 64;
struct BatchIndex {
    int n;                      // entries listed here (0: search the table)
    int first[BATCH_INDEX];
};

__device__ __forceinline__ int batch_entry(const BatchEntry *__restrict__ tab, const BatchIndex &ix, int nshot,
                                           int wg)
{
    int lo = 0, hi = nshot - 1;
    if (ix.n) {
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (ix.first[mid] <= wg) lo = mid;
            else hi = mid - 1;
        }
        return lo;
    }
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab[mid].first <= wg) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int R, bool ADJ>
__global__ __launch_bounds__(TILE_Z * 8)
void step3d_batch_kernel(const BatchEntry *__restrict__ tab, BatchIndex ix, int nshot)
{
    const int s = batch_entry(tab, ix, nshot, blockIdx.x);
    const BatchEntry &e = tab[s];
    step3d_body<R, ADJ, 2>(e.p, blockIdx.x - e.first, e.ntz, e.nty, e.nwg, e.launched);
}

template <int R, bool ADJ>
__global__ __launch_bounds__(TILE_Z2)
void step2d_batch_kernel(const BatchEntry *__restrict__ tab, BatchIndex ix, int nshot)
{
    const int s = batch_entry(tab, ix, nshot, blockIdx.x);
    const BatchEntry &e = tab[s];
    step2d_body<R, ADJ>(e.p, blockIdx.x - e.first, e.ntz, e.nwg);
}

template <int R, bool ADJ>
void launch_r(const StepParams &p, int ndim, hipStream_t st)
{
    BatchEntry e{};
    e.p = p;
    const int total = step_geometry(e, ndim, ADJ);
    if (ndim == 3) {
        if (p.vz == 2) {
            if (p.rpl == 4)
                hipLaunchKernelGGL((step3w_kernel<R, ADJ, 4>), dim3(total), dim3(64, 8, 1), 0, st,
                                   p, e.ntz, e.nty, e.nwg, e.launched);
            else
                hipLaunchKernelGGL((step3w_kernel<R, ADJ, 2>), dim3(total), dim3(64, 8, 1), 0, st,
                                   p, e.ntz, e.nty, e.nwg, e.launched);
        } else if (p.deep)
            hipLaunchKernelGGL((step3d_deep_kernel<R, ADJ>), dim3(total), dim3(TILE_Z, 8, 1), 0, st,
                               p, e.ntz, e.nty, e.nwg, e.launched);
        else if (p.rpl == 4)
            hipLaunchKernelGGL((step3d_kernel<R, ADJ, 4>), dim3(total), dim3(TILE_Z, 8, 1), 0, st,
                               p, e.ntz, e.nty, e.nwg, e.launched);
        else
            hipLaunchKernelGGL((step3d_kernel<R, ADJ, 2>), dim3(total), dim3(TILE_Z, 8, 1), 0, st,
                               p, e.ntz, e.nty, e.nwg, e.launched);
    } else {
        hipLaunchKernelGGL((step2d_kernel<R, ADJ>), dim3(total), dim3(TILE_Z2), 0, st, p, e.ntz, e.nwg);
    }
}

template <int R, bool ADJ>
void launch_batch_r(const BatchEntry *tab, const BatchIndex &ix, int nshot, int total, int ndim, hipStream_t st)
{
    if (ndim == 3)
        hipLaunchKernelGGL((step3d_batch_kernel<R, ADJ>), dim3(total), dim3(TILE_Z, 8, 1), 0, st, tab, ix, nshot);
    else
        hipLaunchKernelGGL((step2d_batch_kernel<R, ADJ>), dim3(total), dim3(TILE_Z2), 0, st, tab, ix, nshot);
}

// ------------------------------------------------------------- small kernels
// Streaming probe: dst_j = sum of the nsrc sources (j < ND), W floats per
// lane per access (4, 8 or 16 bytes), non-temporal loads and stores.  With
// flat = 1 every lane moves one vector and the grid covers the arrays (many
// short workgroups: the fastest streaming form measured on this part);
// otherwise `gridDim.x` workgroups stride over the arrays with four
// accesses per lane in flight.  Measures the practical HBM ceiling of a
// stream mix and serves as the kernel of known traffic for counter
// calibration.
template <int W>
struct VecOf;
template <> struct VecOf<1> { typedef float T; };
template <> struct VecOf<2> { typedef float T __attribute__((ext_vector_type(2))); };
template <> struct VecOf<4> { typedef float T __attribute__((ext_vector_type(4))); };

template <int W, int NS, int ND>
__global__ __launch_bounds__(256) void probe_kernel(ProbeArgs a, int flat)
{
    typedef typename VecOf<W>::T V;
    const size_t nv = a.n / W;
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (flat) {
        if (i >= nv) return;
        V s = __builtin_nontemporal_load(&((const V *)a.src[0])[i]);
#pragma unroll
        for (int k = 1; k < NS; ++k) s += __builtin_nontemporal_load(&((const V *)a.src[k])[i]);
#pragma unroll
        for (int j = 0; j < ND; ++j) __builtin_nontemporal_store(s, &((V *)a.dst[j])[i]);
        return;
    }
    const size_t stride = (size_t)gridDim.x * 256;
    for (; i + 3 * stride < nv; i += 4 * stride) {
        V s[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) s[u] = __builtin_nontemporal_load(&((const V *)a.src[0])[i + u * stride]);
#pragma unroll
        for (int k = 1; k < NS; ++k)
#pragma unroll
            for (int u = 0; u < 4; ++u) s[u] += __builtin_nontemporal_load(&((const V *)a.src[k])[i + u * stride]);
#pragma unroll
        for (int j = 0; j < ND; ++j)
#pragma unroll
            for (int u = 0; u < 4; ++u) __builtin_nontemporal_store(s[u], &((V *)a.dst[j])[i + u * stride]);
    }
    for (; i < nv; i += stride) {
        V s = __builtin_nontemporal_load(&((const V *)a.src[0])[i]);
#pragma unroll
        for (int k = 1; k < NS; ++k) s += __builtin_nontemporal_load(&((const V *)a.src[k])[i]);
#pragma unroll
        for (int j = 0; j < ND; ++j) __builtin_nontemporal_store(s, &((V *)a.dst[j])[i]);
    }
}

// p[0..n) = 0 and dst = src (n floats): kernels rather than memset/memcpy
// nodes, so a captured schedule holds kernel nodes only
__global__ void fill_zero_kernel(float *p, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

__global__ void copy_kernel(float *__restrict__ dst, const float *__restrict__ src, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// b = dt^2/m from the unpadded model into the padded layout
__global__ void coef_kernel(const float *m, float *b, PadMap pm, float dt2)
{
    const size_t n = (size_t)pm.nx * pm.ny * pm.nz;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const size_t z = i % pm.nz, r = i / pm.nz;
        const size_t y = r % pm.ny, x = r / pm.ny;
        b[pm.origin + x * pm.sx + y * pm.sy + z] = dt2 / m[i];
    }
}

// padded (interior only; pads untouched) = unpadded field
__global__ void pad_kernel(const float *f, float *dst, PadMap pm)
{
    const size_t n = (size_t)pm.nx * pm.ny * pm.nz;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const size_t z = i % pm.nz, r = i / pm.nz;
        const size_t y = r % pm.ny, x = r / pm.ny;
        dst[pm.origin + x * pm.sx + y * pm.sy + z] = f[i];
    }
}

// grad (unpadded) = accumulator (padded)
__global__ void unpad_kernel(const float *acc, float *g, PadMap pm)
{
    const size_t n = (size_t)pm.nx * pm.ny * pm.nz;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const size_t z = i % pm.nz, r = i / pm.nz;
        const size_t y = r % pm.ny, x = r / pm.ny;
        g[i] = acc[pm.origin + x * pm.sx + y * pm.sy + z];
    }
}

// one shot's gradient region added into the stacked gradient
__global__ void stack_add_kernel(const float *acc, float *dst, StackMap sm)
{
    const size_t n = (size_t)sm.n[0] * sm.n[1] * sm.n[2];
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const size_t z = i % sm.n[2], r = i / sm.n[2];
        const size_t y = r % sm.n[1], x = r / sm.n[1];
        const size_t src = sm.pm.origin + (sm.r[0] + x) * sm.pm.sx + (sm.r[1] + y) * sm.pm.sy + sm.r[2] + z;
        const size_t d = (sm.o[0] + x) * sm.d0 + (sm.o[1] + y) * sm.d1 + sm.o[2] + z;
        dst[d] += acc[src];
    }
}

__global__ void gather_kernel(const float *f, const int *off, int n, float *out)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = f[off[i]];
}

// r = d_sim - d_obs; per-block FP64 partial sums of r^2 in a fixed order
__global__ __launch_bounds__(256)
void residual_kernel(const float *ds, const float *dob, float *res, size_t n,
                     double *partials)
{
    __shared__ double red[256];
    double acc = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        float r = ds[i] - dob[i];
        res[i] = r;
        acc += (double)r * (double)r;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256)
void phi_kernel(const double *partials, int n, double *phi)
{
    __shared__ double red[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) acc += partials[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *phi = 0.5 * red[0];
}

__device__ __forceinline__ void inject_body(const InjectParams &p, int j)
{
    if (j >= p.nnode) return;
    float s = 0.0f;
    for (int r = p.rec_ptr[j]; r < p.rec_ptr[j + 1]; ++r) s += p.res_row[p.rec_idx[r]];
    const int pi = p.node_pad[j];
    const int x = p.node_xyz[3 * j], y = p.node_xyz[3 * j + 1], z = p.node_xyz[3 * j + 2];
    const int dx = layer_depth(x, p.nx, p.nbl);
    const int dy = p.ndim == 3 ? layer_depth(y, p.ny, p.nbl) : 0;
    const int dz = layer_depth(z, p.nz, p.nbl);
    const float bb = p.b[pi];
    const float e = p.kappa * bb * (float)(dx * dx + dy * dy + dz * dz);
    const float delta = bb * s / (1.0f + e);
    p.lam[pi] += delta;
    if (p.g) p.g[pi] -= p.uk[pi] * delta * p.inv_dt2;
}

__global__ void inject_kernel(InjectParams p)
{
    inject_body(p, blockIdx.x * blockDim.x + threadIdx.x);
}

// every shot of a batched step at once: shot blockIdx.y, table on the device
__global__ void inject_batch_kernel(const InjectParams *__restrict__ tab)
{
    inject_body(tab[blockIdx.y], blockIdx.x * blockDim.x + threadIdx.x);
}

}  // namespace

int step_geometry(BatchEntry &e, int ndim, bool adjoint)
{
    const StepParams &p = e.p;
    const int nchunk = (p.nx + p.xchunk - 1) / p.xchunk;
    const bool gather = !adjoint && p.grow && p.nrec > 0;
    if (ndim == 3) {
        const int rows = 8 * p.rpl;
        const int tzw = p.vz == 2 ? TILE_ZW : TILE_Z;
        e.ntz = (p.nz + tzw - 1) / tzw;
        e.nty = (p.ny + rows - 1) / rows;
        e.nwg = e.ntz * e.nty * nchunk;
        const int unit = p.remap >= 2 ? (8 << (p.remap - 2)) * e.ntz : 8;
        e.launched = ((e.nwg + unit - 1) / unit) * unit;
        const int ng = gather ? (p.nrec + 511) / 512 : 0;
        return e.launched + ng;
    }
    e.ntz = (p.nz + TILE_Z2 - 1) / TILE_Z2;
    e.nty = 1;
    e.nwg = e.ntz * nchunk;
    e.launched = e.nwg;
    const int ng = gather ? (p.nrec + TILE_Z2 - 1) / TILE_Z2 : 0;
    return e.nwg + ng;
}

void launch_step_batch(const BatchEntry *tab, const BatchEntry *host_tab, int nshot, int total, int ndim,
                       int radius, bool adjoint, hipStream_t st)
{
    BatchIndex ix{};
    if (nshot <= BATCH_INDEX) {
        ix.n = nshot;
        for (int i = 0; i < nshot; ++i) ix.first[i] = host_tab[i].first;
    }
    switch (radius * 2 + (adjoint ? 1 : 0)) {
    case 4: launch_batch_r<2, false>(tab, ix, nshot, total, ndim, st); break;
    case 5: launch_batch_r<2, true>(tab, ix, nshot, total, ndim, st); break;
    case 8: launch_batch_r<4, false>(tab, ix, nshot, total, ndim, st); break;
    case 9: launch_batch_r<4, true>(tab, ix, nshot, total, ndim, st); break;
    case 16: launch_batch_r<8, false>(tab, ix, nshot, total, ndim, st); break;
    case 17: launch_batch_r<8, true>(tab, ix, nshot, total, ndim, st); break;
    default: break;
    }
}

void launch_step(const StepParams &p, int ndim, int radius, bool adjoint, hipStream_t st)
{
    switch (radius * 2 + (adjoint ? 1 : 0)) {
    case 4: launch_r<2, false>(p, ndim, st); break;
    case 5: launch_r<2, true>(p, ndim, st); break;
    case 8: launch_r<4, false>(p, ndim, st); break;
    case 9: launch_r<4, true>(p, ndim, st); break;
    case 16: launch_r<8, false>(p, ndim, st); break;
    case 17: launch_r<8, true>(p, ndim, st); break;
    default: break;
    }
}

static int grid_for(size_t n)
{
    size_t blocks = (n + 255) / 256;
    return (int)(blocks > 65536 ? 65536 : blocks);
}

template <int W, int NS>
static void probe_nd(const ProbeArgs &a, int nd, int grid, hipStream_t st)
{
    // grid 0: one vector per lane over the whole arrays
    const int flat = grid == 0;
    const size_t g = flat ? (a.n / W + 255) / 256 : (size_t)grid;
    if (nd == 1) hipLaunchKernelGGL((probe_kernel<W, NS, 1>), dim3((unsigned)g), dim3(256), 0, st, a, flat);
    else hipLaunchKernelGGL((probe_kernel<W, NS, 2>), dim3((unsigned)g), dim3(256), 0, st, a, flat);
}

template <int W>
static void probe_w(const ProbeArgs &a, int ns, int nd, int grid, hipStream_t st)
{
    switch (ns) {
    case 1: probe_nd<W, 1>(a, nd, grid, st); break;
    case 2: probe_nd<W, 2>(a, nd, grid, st); break;
    case 3: probe_nd<W, 3>(a, nd, grid, st); break;
    case 4: probe_nd<W, 4>(a, nd, grid, st); break;
    default: probe_nd<W, 5>(a, nd, grid, st); break;
    }
}

void launch_probe(const ProbeArgs &a, int nsrc, int ndst, int width, int grid, hipStream_t st)
{
    if (width == 16) probe_w<4>(a, nsrc, ndst, grid, st);
    else if (width == 8) probe_w<2>(a, nsrc, ndst, grid, st);
    else probe_w<1>(a, nsrc, ndst, grid, st);
}

void launch_fill_zero(float *p, size_t n, hipStream_t st)
{
    if (n) hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for(n)), dim3(256), 0, st, p, n);
}

void launch_copy(float *dst, const float *src, size_t n, hipStream_t st)
{
    if (n) hipLaunchKernelGGL(copy_kernel, dim3(grid_for(n)), dim3(256), 0, st, dst, src, n);
}

void launch_coef(const float *m, float *b, const PadMap &pm, double dt, hipStream_t st)
{
    hipLaunchKernelGGL(coef_kernel, dim3(grid_for((size_t)pm.nx * pm.ny * pm.nz)), dim3(256), 0, st, m, b,
                       pm, (float)(dt * dt));
}

void launch_unpad(const float *acc, float *g, const PadMap &pm, hipStream_t st)
{
    hipLaunchKernelGGL(unpad_kernel, dim3(grid_for((size_t)pm.nx * pm.ny * pm.nz)), dim3(256), 0, st, acc,
                       g, pm);
}

void launch_stack_add(const float *acc, float *dst, const StackMap &sm, hipStream_t st)
{
    const size_t n = (size_t)sm.n[0] * sm.n[1] * sm.n[2];
    if (n) hipLaunchKernelGGL(stack_add_kernel, dim3(grid_for(n)), dim3(256), 0, st, acc, dst, sm);
}

void launch_pad(const float *f, float *dst, const PadMap &pm, hipStream_t st)
{
    hipLaunchKernelGGL(pad_kernel, dim3(grid_for((size_t)pm.nx * pm.ny * pm.nz)), dim3(256), 0, st, f, dst,
                       pm);
}

void launch_gather(const float *field, const int *off, int n, float *out, hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(gather_kernel, dim3((n + 255) / 256), dim3(256), 0, st, field, off, n, out);
}

void launch_residual(const float *ds, const float *dob, float *res, size_t n,
                     double *partials, int nparts, double *phi, hipStream_t st)
{
    hipLaunchKernelGGL(residual_kernel, dim3(nparts), dim3(256), 0, st, ds, dob, res, n, partials);
    hipLaunchKernelGGL(phi_kernel, dim3(1), dim3(256), 0, st, partials, nparts, phi);
}

void launch_inject(const InjectParams &p, hipStream_t st)
{
    if (p.nnode <= 0) return;
    hipLaunchKernelGGL(inject_kernel, dim3((p.nnode + 127) / 128), dim3(128), 0, st, p);
}

void launch_inject_batch(const InjectParams *dev_tab, int nshot, int max_nodes, hipStream_t st)
{
    if (nshot <= 0 || max_nodes <= 0) return;
    hipLaunchKernelGGL(inject_batch_kernel, dim3((max_nodes + 127) / 128, nshot), dim3(128), 0, st, dev_tab);
}

Padded make_padded(int ndim, const int *comp)
{
    Padded f;
    f.ndim = ndim;
    f.nx = comp[0];
    f.ny = ndim == 3 ? comp[1] : 1;
    f.nz = ndim == 3 ? comp[2] : comp[1];
    f.px = f.nx + 2 * PAD_X;
    const int tz = ndim == 3 ? TILE_ZW : TILE_Z2;
    f.pz = PAD_Z0 + (long)((f.nz + tz - 1) / tz) * tz + PAD_Z0;
    if (ndim == 3) {
        f.py = (long)((f.ny + TILE_Y - 1) / TILE_Y) * TILE_Y + 2 * PAD_Y;
        f.origin = (long)PAD_X * f.py * f.pz + (long)PAD_Y * f.pz + PAD_Z0;
    } else {
        f.py = 1;
        f.origin = (long)PAD_X * f.pz + PAD_Z0;
    }
    f.sy = f.pz;
    f.sx = f.py * f.pz;
    return f;
}

}  // namespace fwi
