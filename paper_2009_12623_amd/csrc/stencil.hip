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
// Work split: a workgroup owns a (y, z) tile (64 z = one wave, TILE_Y waves
// along y; 256 z in 2D) and streams a chunk of x planes.  Each lane keeps the
// 2R+1 x-neighbours of its column in registers; the y and z neighbours of
// the current plane come from an LDS tile whose centre is written from the
// register queue, so global loads per point and step are one new x plane
// value plus the halo ring.  Fields are padded (see internal.hpp), so no
// load needs a bounds check; lanes outside the grid compute nothing.
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

template <int R, bool ADJ>
__device__ __forceinline__ void finish_point(const StepParams &p, int x, int y, int z,
                                             long pi, float c, float lap)
{
    const long ui = (long)x * p.sx + (long)y * p.sy + z;
    const float bb = p.b[ui];
    const float u2v = p.u2[pi];
    const int dx = layer_depth(x, p.nx, p.nbl);
    const int dy = p.ny > 1 ? layer_depth(y, p.ny, p.nbl) : 0;
    const int dz = layer_depth(z, p.nz, p.nbl);
    const int dsum = dx * dx + dy * dy + dz * dz;
    float num;
    float outv;
    if (dsum == 0) {
        num = 2.0f * c + bb * lap - u2v;
        if (!ADJ && ui == p.src) num += bb * p.wav[p.step];
        outv = num;
    } else {
        const float e = p.kappa * bb * (float)dsum;
        num = 2.0f * c + bb * lap - (1.0f - e) * u2v;
        if (!ADJ && ui == p.src) num += bb * p.wav[p.step];
        outv = num / (1.0f + e);
    }
    p.out[pi] = outv;
    if (ADJ) {
        const float ukv = p.uk[pi];
        p.g[ui] -= ukv * (outv - 2.0f * c + u2v) * p.inv_dt2;
    }
}

template <int R, bool ADJ>
__global__ __launch_bounds__(TILE_Z *TILE_Y)
void step3d_kernel(StepParams p)
{
    __shared__ float tile[TILE_Y + 2 * R][TILE_Z + 2 * R];
    const int tz = threadIdx.x;
    const int ty = threadIdx.y;
    const int z0 = blockIdx.x * TILE_Z;
    const int y0 = blockIdx.y * TILE_Y;
    const int z = z0 + tz;
    const int y = y0 + ty;
    const int xb = blockIdx.z * p.xchunk;
    int xe = xb + p.xchunk;
    if (xe > p.nx) xe = p.nx;
    const bool active = z < p.nz && y < p.ny;
    const float *col = p.u1 + (long)y * p.psy + z;

    float q[2 * R + 1];
#pragma unroll
    for (int i = 0; i < 2 * R; ++i) q[i + 1] = col[(long)(xb - R + i) * p.psx];

    for (int x = xb; x < xe; ++x) {
#pragma unroll
        for (int i = 0; i < 2 * R; ++i) q[i] = q[i + 1];
        q[2 * R] = col[(long)(x + R) * p.psx];
        const float *plane = p.u1 + (long)x * p.psx;
        __syncthreads();
        tile[ty + R][tz + R] = q[R];
        for (int r = ty; r < R; r += TILE_Y) {
            tile[r][tz + R] = plane[(long)(y0 - R + r) * p.psy + z];
            tile[r + TILE_Y + R][tz + R] = plane[(long)(y0 + TILE_Y + r) * p.psy + z];
        }
        if (tz < R) tile[ty + R][tz] = plane[(long)y * p.psy + z0 - R + tz];
        if (tz >= TILE_Z - R) tile[ty + R][tz + 2 * R] = plane[(long)y * p.psy + z + R];
        __syncthreads();
        if (active) {
            const float c = q[R];
            float lap = 3.0f * p.w[0] * c;
#pragma unroll
            for (int k = 1; k <= R; ++k)
                lap += p.w[k] * ((q[R - k] + q[R + k]) +
                                 (tile[ty + R - k][tz + R] + tile[ty + R + k][tz + R]) +
                                 (tile[ty + R][tz + R - k] + tile[ty + R][tz + R + k]));
            finish_point<R, ADJ>(p, x, y, z, (long)x * p.psx + (long)y * p.psy + z, c, lap);
        }
    }
}

template <int R, bool ADJ>
__global__ __launch_bounds__(TILE_Z2)
void step2d_kernel(StepParams p)
{
    __shared__ float row[TILE_Z2 + 2 * R];
    const int tz = threadIdx.x;
    const int z0 = blockIdx.x * TILE_Z2;
    const int z = z0 + tz;
    const int xb = blockIdx.z * p.xchunk;
    int xe = xb + p.xchunk;
    if (xe > p.nx) xe = p.nx;
    const bool active = z < p.nz;
    const float *col = p.u1 + z;

    float q[2 * R + 1];
#pragma unroll
    for (int i = 0; i < 2 * R; ++i) q[i + 1] = col[(long)(xb - R + i) * p.psx];

    for (int x = xb; x < xe; ++x) {
#pragma unroll
        for (int i = 0; i < 2 * R; ++i) q[i] = q[i + 1];
        q[2 * R] = col[(long)(x + R) * p.psx];
        const float *line = p.u1 + (long)x * p.psx;
        __syncthreads();
        row[tz + R] = q[R];
        if (tz < R) row[tz] = line[z0 - R + tz];
        if (tz >= TILE_Z2 - R) row[tz + 2 * R] = line[z + R];
        __syncthreads();
        if (active) {
            const float c = q[R];
            float lap = 2.0f * p.w[0] * c;
#pragma unroll
            for (int k = 1; k <= R; ++k)
                lap += p.w[k] * ((q[R - k] + q[R + k]) + (row[tz + R - k] + row[tz + R + k]));
            finish_point<R, ADJ>(p, x, 0, z, (long)x * p.psx + z, c, lap);
        }
    }
}

template <int R, bool ADJ>
void launch_r(const StepParams &p, int ndim, hipStream_t st)
{
    const int nchunk = (p.nx + p.xchunk - 1) / p.xchunk;
    if (ndim == 3) {
        dim3 grid((p.nz + TILE_Z - 1) / TILE_Z, (p.ny + TILE_Y - 1) / TILE_Y, nchunk);
        dim3 block(TILE_Z, TILE_Y, 1);
        hipLaunchKernelGGL((step3d_kernel<R, ADJ>), grid, block, 0, st, p);
    } else {
        dim3 grid((p.nz + TILE_Z2 - 1) / TILE_Z2, 1, nchunk);
        hipLaunchKernelGGL((step2d_kernel<R, ADJ>), grid, dim3(TILE_Z2), 0, st, p);
    }
}

// ------------------------------------------------------------- small kernels
__global__ void coef_kernel(const float *m, float *b, size_t n, float dt2)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n; i += (size_t)gridDim.x * blockDim.x) b[i] = dt2 / m[i];
}

__global__ void gather_kernel(const float *f, const long *off, int n, float *out)
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

__global__ void inject_kernel(InjectParams p)
{
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= p.nnode) return;
    float s = 0.0f;
    for (int r = p.rec_ptr[j]; r < p.rec_ptr[j + 1]; ++r) s += p.res_row[p.rec_idx[r]];
    const long pi = p.node_pad[j];
    const long ui = p.node_unp[j];
    const int x = p.node_xyz[3 * j], y = p.node_xyz[3 * j + 1], z = p.node_xyz[3 * j + 2];
    const int dx = layer_depth(x, p.nx, p.nbl);
    const int dy = p.ndim == 3 ? layer_depth(y, p.ny, p.nbl) : 0;
    const int dz = layer_depth(z, p.nz, p.nbl);
    const float bb = p.b[ui];
    const float e = p.kappa * bb * (float)(dx * dx + dy * dy + dz * dz);
    const float delta = bb * s / (1.0f + e);
    p.lam[pi] += delta;
    p.g[ui] -= p.uk[pi] * delta * p.inv_dt2;
}

}  // namespace

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

void launch_coef(const float *m, float *b, size_t n, double dt, hipStream_t st)
{
    int blocks = (int)((n + 255) / 256);
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(coef_kernel, dim3(blocks), dim3(256), 0, st, m, b, n, (float)(dt * dt));
}

void launch_gather(const float *field, const long *off, int n, float *out, hipStream_t st)
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

Padded make_padded(int ndim, const int *comp)
{
    Padded f;
    f.ndim = ndim;
    f.nx = comp[0];
    f.ny = ndim == 3 ? comp[1] : 1;
    f.nz = ndim == 3 ? comp[2] : comp[1];
    f.px = f.nx + 2 * PAD_X;
    const int tz = ndim == 3 ? TILE_Z : TILE_Z2;
    f.pz = PAD_Z0 + (long)((f.nz + tz - 1) / tz) * tz + 16;
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
