// kbc_kernels.hip -- gfx950 kernels of the D3Q27 KBC lattice Boltzmann box
// other than the step itself (kbc_step.h, instantiated in kbc_step_inst.hip):
// initialisation at the product-form equilibrium, layout conversion, FP64
// diagnostics, the streaming copy, and the launchers of all of them.
#include <hip/hip_runtime.h>
#include <math.h>

#include "kbc_device.h"
#include "kbc_internal.h"
#include "kbc_step.h"

namespace kbc {

namespace {

template <int S>
__device__ __forceinline__ void store_full(void* buf, uint64_t idx, int slot, int i,
                                           const float* scale, double f)
{
    using T = typename Traits<S>::T;
    T* b = static_cast<T*>(buf);
    if constexpr (S == ST_F64) b[idx] = f;
    else if constexpr (S == ST_F32) b[idx] = (float)(f - weight(i));
    else b[idx] = (_Float16)((float)(f - weight(i)) * scale[slot]);
}

// Product-form equilibrium of section II through its one-dimensional
// marginals, in FP64: e_0 = (4 - 2S)/3, e_{+-1} = ((2S - 1)/3 +- u)/2.
__device__ __forceinline__ void marginals(double u, double e[3])
{
    const double q3 = 3.0 * u * u;
    const double sm1 = q3 / (1.0 + sqrt(1.0 + q3));
    e[1] = 2.0 / 3.0 - (2.0 / 3.0) * sm1;
    e[2] = 1.0 / 6.0 + sm1 / 3.0 + 0.5 * u;
    e[0] = 1.0 / 6.0 + sm1 / 3.0 - 0.5 * u;
}

struct StoreCtx {
    float scale[27];
};

template <int S>
__global__ void __launch_bounds__(kBlock) k_init_feq(int layout, void* buf, Geom g, StoreCtx sc,
                                                     const double* __restrict__ u,
                                                     const double* __restrict__ rho)
{
    const uint32_t n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.nnodes) return;
    uint32_t x, y, z;
    node_xyz(n, g, x, y, z);
    const double r = rho ? rho[n] : 1.0;
    double ex[3], ey[3], ez[3];
    marginals(u[n], ex);
    marginals(u[g.nnodes + n], ey);
    marginals(u[2 * (size_t)g.nnodes + n], ez);
    for (int i = 0; i < 27; ++i) {
        const double feq = r * ex[i % 3] * ey[(i / 3) % 3] * ez[i / 9];
        int slot;
        const uint64_t idx = locate(layout, i, x, y, z, g, slot);
        store_full<S>(buf, idx, slot, i, sc.scale, feq);
    }
}

__global__ void __launch_bounds__(kBlock) k_check_init(Geom g, const double* __restrict__ u,
                                                       const double* __restrict__ rho, int* flag)
{
    const uint32_t n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.nnodes) return;
    bool bad = false;
    for (int a = 0; a < 3; ++a) {
        const double v = u[a * (size_t)g.nnodes + n];
        bad |= !(fabs(v) < 1.0);
    }
    if (rho) bad |= !(rho[n] > 0.0 && isfinite(rho[n]));
    if (bad) atomicOr(flag, 1);
}

// Per-direction maximum over the block first (non-negative floats compare
// like their bit patterns), then one atomic per direction and block.
__device__ __forceinline__ void block_max_27(float (&d)[27], unsigned* max_bits)
{
    __shared__ unsigned red[27];
    if (threadIdx.x < 27) red[threadIdx.x] = 0u;
    __syncthreads();
    for (int i = 0; i < 27; ++i) {
        unsigned v = __float_as_uint(d[i]);
        for (int off = 32; off > 0; off >>= 1) v = max(v, (unsigned)__shfl_xor((int)v, off, 64));
        if ((threadIdx.x & 63) == 0) atomicMax(&red[i], v);
    }
    __syncthreads();
    if (threadIdx.x < 27) atomicMax(&max_bits[threadIdx.x], red[threadIdx.x]);
}

__global__ void __launch_bounds__(kBlock) k_feq_dev_max(Geom g, const double* __restrict__ u,
                                                        const double* __restrict__ rho,
                                                        unsigned* max_bits)
{
    const uint32_t n = blockIdx.x * kBlock + threadIdx.x;
    float d[27];
    for (int i = 0; i < 27; ++i) d[i] = 0.0f;
    if (n < g.nnodes) {
        const double r = rho ? rho[n] : 1.0;
        double ex[3], ey[3], ez[3];
        marginals(u[n], ex);
        marginals(u[g.nnodes + n], ey);
        marginals(u[2 * (size_t)g.nnodes + n], ez);
        for (int i = 0; i < 27; ++i)
            d[i] = (float)fabs(r * ex[i % 3] * ey[(i / 3) % 3] * ez[i / 9] - weight(i));
    }
    block_max_27(d, max_bits);
}

__global__ void __launch_bounds__(kBlock) k_pop_dev_max(Geom g, const double* __restrict__ f,
                                                        unsigned* max_bits)
{
    const uint32_t n = blockIdx.x * kBlock + threadIdx.x;
    float d[27];
    for (int i = 0; i < 27; ++i)
        d[i] = n < g.nnodes ? (float)fabs(f[i * (size_t)g.nnodes + n] - weight(i)) : 0.0f;
    block_max_27(d, max_bits);
}

template <int S>
__global__ void __launch_bounds__(kBlock) k_gather_pop(int layout, const void* buf, Geom g,
                                                       LoadCtx lc, double* __restrict__ f)
{
    const uint32_t n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.nnodes) return;
    uint32_t x, y, z;
    node_xyz(n, g, x, y, z);
    for (int i = 0; i < 27; ++i) {
        int slot;
        const uint64_t idx = locate(layout, i, x, y, z, g, slot);
        f[i * (size_t)g.nnodes + n] = load_full<S>(buf, idx, slot, i, lc.inv_scale);
    }
}

template <int S>
__global__ void __launch_bounds__(kBlock) k_sample_pop(int layout, const void* buf, Geom g,
                                                       LoadCtx lc, const uint32_t* __restrict__ nodes,
                                                       int count, double* __restrict__ out)
{
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= count) return;
    const uint32_t n = nodes[k];
    uint32_t x, y, z;
    node_xyz(n, g, x, y, z);
    for (int i = 0; i < 27; ++i) {
        int slot;
        const uint64_t idx = locate(layout, i, x, y, z, g, slot);
        out[27 * (size_t)k + i] = load_full<S>(buf, idx, slot, i, lc.inv_scale);
    }
}

template <int S>
__global__ void __launch_bounds__(kBlock) k_scatter_pop(int layout, void* buf, Geom g, StoreCtx sc,
                                                        const double* __restrict__ f)
{
    const uint32_t n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.nnodes) return;
    uint32_t x, y, z;
    node_xyz(n, g, x, y, z);
    for (int i = 0; i < 27; ++i) {
        int slot;
        const uint64_t idx = locate(layout, i, x, y, z, g, slot);
        store_full<S>(buf, idx, slot, i, sc.scale, f[i * (size_t)g.nnodes + n]);
    }
}

// rho = sum_i f_i, rho u = sum_i v_i f_i (section I) of node n, in FP64.
// Deviation forms sum the stored deviations and add the weights' share
// (1, 0).  Every kernel that needs the velocity of F(t) takes it from here,
// so they all see the same bits.
template <int S>
__device__ __forceinline__ void node_velocity(int layout, const void* buf, const Geom& g,
                                              const LoadCtx& lc, uint32_t n, double& m,
                                              double& ux, double& uy, double& uz)
{
    uint32_t x, y, z;
    node_xyz(n, g, x, y, z);
    double jx = 0.0, jy = 0.0, jz = 0.0;
    m = 0.0;
    for (int i = 0; i < 27; ++i) {
        int slot;
        const uint64_t idx = locate(layout, i, x, y, z, g, slot);
        double v = load_full<S>(buf, idx, slot, i, lc.inv_scale);
        if constexpr (S != ST_F64) v -= weight(i);
        m += v;
        jx += vel(i, 0) * v;
        jy += vel(i, 1) * v;
        jz += vel(i, 2) * v;
    }
    if constexpr (S != ST_F64) m += 1.0;
    const double ir = 1.0 / m;
    ux = jx * ir;
    uy = jy * ir;
    uz = jz * ir;
}

template <int S>
__global__ void __launch_bounds__(kBlock) k_moments(int layout, const void* buf, Geom g, LoadCtx lc,
                                                    double* __restrict__ rho,
                                                    double* __restrict__ u, int* flag)
{
    const uint32_t n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.nnodes) return;
    double m, ux, uy, uz;
    node_velocity<S>(layout, buf, g, lc, n, m, ux, uy, uz);
    if (rho) rho[n] = m;
    u[n] = ux;
    u[g.nnodes + n] = uy;
    u[2 * (size_t)g.nnodes + n] = uz;
    if (!(isfinite(m) && isfinite(ux) && isfinite(uy) && isfinite(uz))) atomicOr(flag, 1);
}

// ---------------------------------------------------------------------------
// Deterministic FP64 reductions: fixed grid, fixed per-thread order,
// butterfly within the wavefront, fixed order across wavefronts and blocks.
// ---------------------------------------------------------------------------
constexpr int kReduceBlocks = 1024;
template <int KIND>
__global__ void __launch_bounds__(kBlock) k_reduce(Geom g, const double* __restrict__ u,
                                                   const double* __restrict__ mean_sum,
                                                   double* __restrict__ partial)
{
    const size_t N = g.nnodes;
    double acc[3] = {0.0, 0.0, 0.0};
    double mean[3] = {0.0, 0.0, 0.0};
    if (KIND != 0)
        for (int a = 0; a < 3; ++a) mean[a] = mean_sum[a] / (double)N;
    for (uint32_t n = blockIdx.x * kBlock + threadIdx.x; n < g.nnodes; n += gridDim.x * kBlock) {
        if (KIND == 0) {
            for (int a = 0; a < 3; ++a) acc[a] += u[a * N + n];
        } else if (KIND == 1) {
            for (int a = 0; a < 3; ++a) {
                const double d = u[a * N + n] - mean[a];
                acc[0] += d * d;
            }
        } else {
            uint32_t x, y, z;
            node_xyz(n, g, x, y, z);
            const uint32_t xp = node_of(wrap_add(x, 1, g.nx), y, z, g);
            const uint32_t xm = node_of(wrap_add(x, -1, g.nx), y, z, g);
            const uint32_t yp = node_of(x, wrap_add(y, 1, g.ny), z, g);
            const uint32_t ym = node_of(x, wrap_add(y, -1, g.ny), z, g);
            const uint32_t zp = node_of(x, y, wrap_add(z, 1, g.nz), g);
            const uint32_t zm = node_of(x, y, wrap_add(z, -1, g.nz), g);
            auto up = [&](int a, uint32_t m) { return u[a * N + m] - mean[a]; };
            const double wx = 0.5 * (up(2, yp) - up(2, ym)) - 0.5 * (up(1, zp) - up(1, zm));
            const double wy = 0.5 * (up(0, zp) - up(0, zm)) - 0.5 * (up(2, xp) - up(2, xm));
            const double wz = 0.5 * (up(1, xp) - up(1, xm)) - 0.5 * (up(0, yp) - up(0, ym));
            acc[0] += wx * wx + wy * wy + wz * wz;
        }
    }
    block_sum<3>(acc, partial + 3 * blockIdx.x);
}

__global__ void __launch_bounds__(kBlock) k_reduce_final(const double* __restrict__ partial,
                                                         int count, double* __restrict__ out)
{
    double acc[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < count; b += kBlock)
        for (int k = 0; k < 3; ++k) acc[k] += partial[3 * b + k];
    block_sum<3>(acc, out);
}

// Kinetic energy straight from the populations, without a velocity field in
// memory: pass 0 sums u over the nodes, pass 1 sums |u - mean|^2 (mean =
// mean_sum / N).  The grid, the per-thread order and the block reduction are
// those of k_reduce over a stored field, and u comes from node_velocity as in
// k_moments, so the sums are the same bits as moments + k_reduce.
template <int S, int PASS>
__global__ void __launch_bounds__(kBlock) k_energy_pass(int layout, const void* buf, Geom g,
                                                        LoadCtx lc,
                                                        const double* __restrict__ mean_sum,
                                                        double* __restrict__ partial)
{
    const size_t N = g.nnodes;
    double acc[3] = {0.0, 0.0, 0.0};
    double mean[3] = {0.0, 0.0, 0.0};
    if (PASS != 0)
        for (int a = 0; a < 3; ++a) mean[a] = mean_sum[a] / (double)N;
    for (uint32_t n = blockIdx.x * kBlock + threadIdx.x; n < g.nnodes; n += gridDim.x * kBlock) {
        double m, uu[3];
        node_velocity<S>(layout, buf, g, lc, n, m, uu[0], uu[1], uu[2]);
        // u as k_moments stores it: rounded, not fused into u - mean below
        asm volatile("" : "+v"(uu[0]), "+v"(uu[1]), "+v"(uu[2]));
        if (PASS == 0) {
            for (int a = 0; a < 3; ++a) acc[a] += uu[a];
        } else {
            for (int a = 0; a < 3; ++a) {
                const double d = uu[a] - mean[a];
                acc[0] += d * d;
            }
        }
    }
    block_sum<3>(acc, partial + 3 * blockIdx.x);
}

// First component of k_reduce_final only (same order, same bits), for a
// destination with room for one value.
__global__ void __launch_bounds__(kBlock) k_reduce_final_1(const double* __restrict__ partial,
                                                           int count, double* __restrict__ out)
{
    double acc[1] = {0.0};
    for (int b = threadIdx.x; b < count; b += kBlock) acc[0] += partial[3 * b];
    block_sum<1>(acc, out);
}

template <int K>
__global__ void __launch_bounds__(kBlock) k_reduce_final_k(const double* __restrict__ partial,
                                                           int count, double* __restrict__ out)
{
    double acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.0;
    for (int b = threadIdx.x; b < count; b += kBlock)
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] += partial[K * b + k];
    block_sum<K>(acc, out);
}

// ---------------------------------------------------------------------------
// Flow statistics of section V from the velocity field u[3][N].
// ---------------------------------------------------------------------------

// (a + d) mod n for any small signed d
__device__ __forceinline__ uint32_t wrap_mod(uint32_t a, int d, uint32_t n)
{
    int64_t v = ((int64_t)a + d) % (int64_t)n;
    return (uint32_t)(v < 0 ? v + n : v);
}

// Central first-derivative weights of f(x+m) - f(x-m): second order, and
// the nine-point eighth-order stencil.
template <int ORD> struct FdW;
template <> struct FdW<2> {
    static constexpr int M = 1;
    __device__ static constexpr double c(int) { return 0.5; }
};
template <> struct FdW<8> {
    static constexpr int M = 4;
    __device__ static constexpr double c(int m)
    {
        return m == 1 ? 4.0 / 5.0 : (m == 2 ? -1.0 / 5.0 : (m == 3 ? 4.0 / 105.0 : -1.0 / 280.0));
    }
};

// Per-block sums of |curl u|^2, sum_ab (d_a u_b + d_b u_a)^2, (div u)^2 and
// (du_x/dx)^n for n = 2..6 (grid-stride, fixed order).
template <int ORD>
__global__ void __launch_bounds__(kBlock) k_grad_stats(Geom g, const double* __restrict__ u,
                                                       double* __restrict__ partial)
{
    const size_t N = g.nnodes;
    double acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = 0.0;
    for (uint32_t n = blockIdx.x * kBlock + threadIdx.x; n < g.nnodes; n += gridDim.x * kBlock) {
        uint32_t x, y, z;
        node_xyz(n, g, x, y, z);
        double G[3][3];  // G[a][b] = d u_a / d x_b
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            uint32_t np[FdW<ORD>::M], nm[FdW<ORD>::M];
#pragma unroll
            for (int m = 1; m <= FdW<ORD>::M; ++m) {
                if (b == 0) {
                    np[m - 1] = node_of(wrap_mod(x, m, g.nx), y, z, g);
                    nm[m - 1] = node_of(wrap_mod(x, -m, g.nx), y, z, g);
                } else if (b == 1) {
                    np[m - 1] = node_of(x, wrap_mod(y, m, g.ny), z, g);
                    nm[m - 1] = node_of(x, wrap_mod(y, -m, g.ny), z, g);
                } else {
                    np[m - 1] = node_of(x, y, wrap_mod(z, m, g.nz), g);
                    nm[m - 1] = node_of(x, y, wrap_mod(z, -m, g.nz), g);
                }
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                double d = 0.0;
#pragma unroll
                for (int m = 1; m <= FdW<ORD>::M; ++m)
                    d += FdW<ORD>::c(m) * (u[a * N + np[m - 1]] - u[a * N + nm[m - 1]]);
                G[a][b] = d;
            }
        }
        const double wx = G[2][1] - G[1][2], wy = G[0][2] - G[2][0], wz = G[1][0] - G[0][1];
        acc[0] += wx * wx + wy * wy + wz * wz;
        double e = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const double sab = G[a][b] + G[b][a];
                e += sab * sab;
            }
        acc[1] += e;
        const double dv = G[0][0] + G[1][1] + G[2][2];
        acc[2] += dv * dv;
        const double d1 = G[0][0], d2 = d1 * d1, d3 = d2 * d1;
        acc[3] += d2;
        acc[4] += d3;
        acc[5] += d2 * d2;
        acc[6] += d3 * d2;
        acc[7] += d3 * d3;
    }
    block_sum<8>(acc, partial + 8 * blockIdx.x);
}


__global__ void __launch_bounds__(kBlock) k_gamma_final(const double* __restrict__ partial,
                                                        int count, double* __restrict__ out)
{
    double acc[2] = {0.0, 0.0};
    double lo = __builtin_inf(), hi = -__builtin_inf();
    for (int b = threadIdx.x; b < count; b += kBlock) {
        acc[0] += partial[4 * b];
        acc[1] += partial[4 * b + 1];
        lo = fmin(lo, partial[4 * b + 2]);
        hi = fmax(hi, partial[4 * b + 3]);
    }
    double tmp[2];
    block_sum<2>(acc, tmp);  // thread 0 holds the sums in tmp
    __shared__ double mn[kBlock / 64], mx[kBlock / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, off, 64));
        hi = fmax(hi, __shfl_xor(hi, off, 64));
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        mn[wave] = lo;
        mx[wave] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 0; w < kBlock / 64; ++w) {
            lo = fmin(lo, mn[w]);
            hi = fmax(hi, mx[w]);
        }
        out[0] = tmp[0];
        out[1] = tmp[1];
        out[2] = lo;
        out[3] = hi;
    }
}

// Sums over the (y, z) lines of u'_c(x) u'_c(x + r) for c = x, y components
// and r = 0..rmax.  A block stages one line at a time in LDS; thread t owns
// the lags r = t, t + kBlock, ... (at most kCorrLags per thread) for all the
// lines the block visits, so the per-block sums come out in a fixed order.
constexpr int kCorrLags = 8;
constexpr int kCorrMaxN = 4096;

__global__ void __launch_bounds__(kBlock) k_corr_x(Geom g, const double* __restrict__ u,
                                                   const double* __restrict__ mean_sum, int rmax,
                                                   double* __restrict__ partial)
{
    __shared__ double line[2][kCorrMaxN];
    const size_t N = g.nnodes;
    const double mx = mean_sum[0] / (double)N, my = mean_sum[1] / (double)N;
    double acc[2][kCorrLags];
#pragma unroll
    for (int k = 0; k < kCorrLags; ++k) acc[0][k] = acc[1][k] = 0.0;
    const uint32_t lines = g.ny * g.nz;
    for (uint32_t l = blockIdx.x; l < lines; l += gridDim.x) {
        const size_t base = (size_t)l * g.nx;
        __syncthreads();
        for (uint32_t x = threadIdx.x; x < g.nx; x += kBlock) {
            line[0][x] = u[base + x] - mx;
            line[1][x] = u[N + base + x] - my;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kCorrLags; ++k) {
            const int r = threadIdx.x + k * kBlock;
            if (r > rmax) break;
            double s0 = 0.0, s1 = 0.0;
            uint32_t xr = (uint32_t)r % g.nx;
            for (uint32_t x = 0; x < g.nx; ++x) {
                s0 += line[0][x] * line[0][xr];
                s1 += line[1][x] * line[1][xr];
                xr = xr + 1 == g.nx ? 0u : xr + 1;
            }
            acc[0][k] += s0;
            acc[1][k] += s1;
        }
    }
    const int L = rmax + 1;
#pragma unroll
    for (int k = 0; k < kCorrLags; ++k) {
        const int r = threadIdx.x + k * kBlock;
        if (r < L) {
            partial[((size_t)blockIdx.x * L + r) * 2] = acc[0][k];
            partial[((size_t)blockIdx.x * L + r) * 2 + 1] = acc[1][k];
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_corr_final(const double* __restrict__ partial,
                                                       int blocks, int rmax, double* __restrict__ out)
{
    const int L = rmax + 1;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= 2 * L) return;
    double s = 0.0;
    for (int b = 0; b < blocks; ++b) s += partial[(size_t)b * 2 * L + t];
    out[t] = s;  // out[2r + c]
}

inline unsigned grid_for(uint32_t n) { return (n + kBlock - 1) / kBlock; }

__global__ void k_zero_u32(unsigned* p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Streaming copy: one 16-byte word per thread and iteration (ordinary
// loads, non-temporal stores); the grid covers up to 2^21 blocks, which is
// the whole array for copies up to 8 GiB.  This form measured fastest among
// the copies tried (16 B or 8 B per lane, 1 or 4 words per thread, with or
// without non-temporal loads).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(kBlock) k_copy16(u32x4* __restrict__ dst,
                                                  const u32x4* __restrict__ src, size_t n16)
{
    const size_t stride = (size_t)gridDim.x * kBlock;
    for (size_t k = (size_t)blockIdx.x * kBlock + threadIdx.x; k < n16; k += stride)
        __builtin_nontemporal_store(src[k], &dst[k]);
}

// The same stream in place: every 16-byte word is read and written back to
// its own address, the access pattern of an in-place sweep.  `mask` is zero
// at run time (the data stays as it was); XOR-ing it into all four lanes
// keeps the compiler from dropping (or narrowing) the store of a value just
// loaded from the same address.
__global__ void __launch_bounds__(kBlock) k_rewrite16(u32x4* p, size_t n16, uint32_t mask)
{
    const size_t stride = (size_t)gridDim.x * kBlock;
    for (size_t k = (size_t)blockIdx.x * kBlock + threadIdx.x; k < n16; k += stride) {
        u32x4 v = p[k];
        v ^= mask;
        __builtin_nontemporal_store(v, &p[k]);
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t step_launch_shape(int storage, int variant, int sweep, bool exact_gamma, const Geom& g,
                             StepFn* fn, uint32_t* grid, uint32_t* block)
{
    // the AA kernels address populations in planes (see node_update)
    if (sweep != SW_PULL && !geom_is_planes(g)) return hipErrorInvalidValue;
    // x-blocked in chunks of 64 nodes (geom_blocked)
    const bool c64 = g.xshift == 6 && g.xmask == 63 && g.plane == 64 && g.chunk == 27 * 64;
    switch (storage) {
    case ST_F64: *fn = exact_gamma ? step_kernel<ST_F64, true>(variant, sweep, c64) : step_kernel<ST_F64, false>(variant, sweep, c64); break;
    case ST_F32: *fn = exact_gamma ? step_kernel<ST_F32, true>(variant, sweep, c64) : step_kernel<ST_F32, false>(variant, sweep, c64); break;
    case ST_F32X: *fn = exact_gamma ? step_kernel<ST_F32X, true>(variant, sweep, c64) : step_kernel<ST_F32X, false>(variant, sweep, c64); break;
    default: *fn = exact_gamma ? step_kernel<ST_F16, true>(variant, sweep, c64) : step_kernel<ST_F16, false>(variant, sweep, c64); break;
    }
    // One wavefront per workgroup for the exact stabilizer (one wave per
    // SIMD: 64-thread workgroups fill the CUs more evenly; at 256^3 the pull
    // sweep ran 14% (FP64) and 5% (FP32-X) faster than with 256 threads, the
    // AA sweeps 12% and 8%), kStepBlock threads otherwise (64 measured within
    // +-2% for the other pull forms, 5% slower for FP16 pull, and 17-33%
    // slower for the AA sweeps).
    *block = exact_gamma ? 64u : (uint32_t)kStepBlock;
    *grid = (g.nnodes + *block - 1) / *block;
    return hipSuccess;
}

hipError_t launch_step(int storage, int variant, int sweep, bool exact_gamma, const StepParams& p,
                       hipStream_t stream)
{
    StepFn fn;
    uint32_t grid, block;
    hipError_t e = step_launch_shape(storage, variant, sweep, exact_gamma, p.g, &fn, &grid, &block);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(block), 0, stream, p);
    return hipGetLastError();
}

hipError_t launch_pool_step(int storage, int variant, int sweep, const PoolBox* boxes,
                            const uint32_t* tstart, const PoolMeta* meta, int k, int block,
                            int grid, bool one, hipStream_t stream)
{
    if (block < 64 || block > kPoolMaxBlock || block % 64 || grid < 1) return hipErrorInvalidValue;
    if (sweep != SW_AA_EVEN && sweep != SW_AA_ODD) return hipErrorInvalidValue;
    PoolFn fn;
    switch (storage) {
    case ST_F64: fn = pool_kernel<ST_F64>(variant, sweep, one); break;
    case ST_F32: fn = pool_kernel<ST_F32>(variant, sweep, one); break;
    case ST_F32X: fn = pool_kernel<ST_F32X>(variant, sweep, one); break;
    default: fn = pool_kernel<ST_F16>(variant, sweep, one); break;
    }
    hipLaunchKernelGGL(fn, dim3(grid), dim3(block), 0, stream, boxes, tstart, meta, k);
    return hipGetLastError();
}

hipError_t launch_init_feq(int storage, int layout, void* buf, const Geom& g, const float* scale,
                           const double* u, const double* rho, hipStream_t stream)
{
    if (storage == ST_F32X) storage = ST_F32;  // same storage format
    StoreCtx sc;
    for (int i = 0; i < 27; ++i) sc.scale[i] = scale ? scale[i] : 1.0f;
    const dim3 grid(grid_for(g.nnodes)), block(kBlock);
    if (storage == ST_F64) hipLaunchKernelGGL(k_init_feq<ST_F64>, grid, block, 0, stream, layout, buf, g, sc, u, rho);
    else if (storage == ST_F32) hipLaunchKernelGGL(k_init_feq<ST_F32>, grid, block, 0, stream, layout, buf, g, sc, u, rho);
    else hipLaunchKernelGGL(k_init_feq<ST_F16>, grid, block, 0, stream, layout, buf, g, sc, u, rho);
    return hipGetLastError();
}

hipError_t launch_check_init(const Geom& g, const double* u, const double* rho, int* flag,
                             hipStream_t stream)
{
    hipLaunchKernelGGL(k_check_init, dim3(grid_for(g.nnodes)), dim3(kBlock), 0, stream, g, u, rho, flag);
    return hipGetLastError();
}

hipError_t launch_feq_dev_max(const Geom& g, const double* u, const double* rho, unsigned* max_bits,
                              hipStream_t stream)
{
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, stream, max_bits, 27);
    hipLaunchKernelGGL(k_feq_dev_max, dim3(grid_for(g.nnodes)), dim3(kBlock), 0, stream, g, u, rho, max_bits);
    return hipGetLastError();
}

hipError_t launch_pop_dev_max(const Geom& g, const double* f, unsigned* max_bits, hipStream_t stream)
{
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, stream, max_bits, 27);
    hipLaunchKernelGGL(k_pop_dev_max, dim3(grid_for(g.nnodes)), dim3(kBlock), 0, stream, g, f, max_bits);
    return hipGetLastError();
}

hipError_t launch_gather_pop(int storage, int layout, const void* buf, const Geom& g,
                             const float* inv_scale, double* f, hipStream_t stream)
{
    if (storage == ST_F32X) storage = ST_F32;  // same storage format
    LoadCtx lc;
    for (int i = 0; i < 27; ++i) lc.inv_scale[i] = inv_scale ? inv_scale[i] : 1.0f;
    const dim3 grid(grid_for(g.nnodes)), block(kBlock);
    if (storage == ST_F64) hipLaunchKernelGGL(k_gather_pop<ST_F64>, grid, block, 0, stream, layout, buf, g, lc, f);
    else if (storage == ST_F32) hipLaunchKernelGGL(k_gather_pop<ST_F32>, grid, block, 0, stream, layout, buf, g, lc, f);
    else hipLaunchKernelGGL(k_gather_pop<ST_F16>, grid, block, 0, stream, layout, buf, g, lc, f);
    return hipGetLastError();
}

hipError_t launch_sample_pop(int storage, int layout, const void* buf, const Geom& g,
                             const float* inv_scale, const uint32_t* nodes, int count,
                             double* out, hipStream_t stream)
{
    if (storage == ST_F32X) storage = ST_F32;  // same storage format
    LoadCtx lc;
    for (int i = 0; i < 27; ++i) lc.inv_scale[i] = inv_scale ? inv_scale[i] : 1.0f;
    const dim3 grid((count + kBlock - 1) / kBlock), block(kBlock);
    if (storage == ST_F64) hipLaunchKernelGGL(k_sample_pop<ST_F64>, grid, block, 0, stream, layout, buf, g, lc, nodes, count, out);
    else if (storage == ST_F32) hipLaunchKernelGGL(k_sample_pop<ST_F32>, grid, block, 0, stream, layout, buf, g, lc, nodes, count, out);
    else hipLaunchKernelGGL(k_sample_pop<ST_F16>, grid, block, 0, stream, layout, buf, g, lc, nodes, count, out);
    return hipGetLastError();
}

hipError_t launch_scatter_pop(int storage, int layout, void* buf, const Geom& g, const float* scale,
                              const double* f, hipStream_t stream)
{
    if (storage == ST_F32X) storage = ST_F32;  // same storage format
    StoreCtx sc;
    for (int i = 0; i < 27; ++i) sc.scale[i] = scale ? scale[i] : 1.0f;
    const dim3 grid(grid_for(g.nnodes)), block(kBlock);
    if (storage == ST_F64) hipLaunchKernelGGL(k_scatter_pop<ST_F64>, grid, block, 0, stream, layout, buf, g, sc, f);
    else if (storage == ST_F32) hipLaunchKernelGGL(k_scatter_pop<ST_F32>, grid, block, 0, stream, layout, buf, g, sc, f);
    else hipLaunchKernelGGL(k_scatter_pop<ST_F16>, grid, block, 0, stream, layout, buf, g, sc, f);
    return hipGetLastError();
}

hipError_t launch_moments(int storage, int layout, const void* buf, const Geom& g,
                          const float* inv_scale, double* rho, double* u, int* flag,
                          hipStream_t stream)
{
    if (storage == ST_F32X) storage = ST_F32;  // same storage format
    LoadCtx lc;
    for (int i = 0; i < 27; ++i) lc.inv_scale[i] = inv_scale ? inv_scale[i] : 1.0f;
    const dim3 grid(grid_for(g.nnodes)), block(kBlock);
    if (storage == ST_F64) hipLaunchKernelGGL(k_moments<ST_F64>, grid, block, 0, stream, layout, buf, g, lc, rho, u, flag);
    else if (storage == ST_F32) hipLaunchKernelGGL(k_moments<ST_F32>, grid, block, 0, stream, layout, buf, g, lc, rho, u, flag);
    else hipLaunchKernelGGL(k_moments<ST_F16>, grid, block, 0, stream, layout, buf, g, lc, rho, u, flag);
    return hipGetLastError();
}

hipError_t launch_copy16(void* dst, const void* src, size_t n16, hipStream_t stream)
{
    if (n16 == 0) return hipSuccess;
    const size_t want = (n16 + kBlock - 1) / kBlock;
    const unsigned blocks = (unsigned)std::min<size_t>(want, 1u << 21);
    hipLaunchKernelGGL(k_copy16, dim3(blocks), dim3(kBlock), 0, stream, static_cast<u32x4*>(dst),
                       static_cast<const u32x4*>(src), n16);
    return hipGetLastError();
}

hipError_t launch_rewrite16(void* p, size_t n16, hipStream_t stream)
{
    if (n16 == 0) return hipSuccess;
    const size_t want = (n16 + kBlock - 1) / kBlock;
    const unsigned blocks = (unsigned)std::min<size_t>(want, 1u << 21);
    hipLaunchKernelGGL(k_rewrite16, dim3(blocks), dim3(kBlock), 0, stream, static_cast<u32x4*>(p),
                       n16, 0u);
    return hipGetLastError();
}

int reduce_partials() { return kReduceBlocks; }

hipError_t launch_reduce(int kind, const Geom& g, const double* u, const double* mean_sum,
                         double* partial, double* out, hipStream_t stream)
{
    const unsigned blocks = std::min<unsigned>(kReduceBlocks, grid_for(g.nnodes));
    if (kind == 0) hipLaunchKernelGGL(k_reduce<0>, dim3(blocks), dim3(kBlock), 0, stream, g, u, mean_sum, partial);
    else if (kind == 1) hipLaunchKernelGGL(k_reduce<1>, dim3(blocks), dim3(kBlock), 0, stream, g, u, mean_sum, partial);
    else hipLaunchKernelGGL(k_reduce<2>, dim3(blocks), dim3(kBlock), 0, stream, g, u, mean_sum, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kBlock), 0, stream, partial, (int)blocks, out);
    return hipGetLastError();
}

hipError_t launch_energy_direct(int storage, int layout, const void* buf, const Geom& g,
                                const float* inv_scale, double* partial, double* sums,
                                double* out, hipStream_t stream)
{
    if (storage == ST_F32X) storage = ST_F32;  // same storage format
    LoadCtx lc;
    for (int i = 0; i < 27; ++i) lc.inv_scale[i] = inv_scale ? inv_scale[i] : 1.0f;
    const unsigned blocks = std::min<unsigned>(kReduceBlocks, grid_for(g.nnodes));
    const dim3 grid(blocks), block(kBlock);
    if (storage == ST_F64) hipLaunchKernelGGL((k_energy_pass<ST_F64, 0>), grid, block, 0, stream, layout, buf, g, lc, sums, partial);
    else if (storage == ST_F32) hipLaunchKernelGGL((k_energy_pass<ST_F32, 0>), grid, block, 0, stream, layout, buf, g, lc, sums, partial);
    else hipLaunchKernelGGL((k_energy_pass<ST_F16, 0>), grid, block, 0, stream, layout, buf, g, lc, sums, partial);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kBlock), 0, stream, partial, (int)blocks, sums);
    if (storage == ST_F64) hipLaunchKernelGGL((k_energy_pass<ST_F64, 1>), grid, block, 0, stream, layout, buf, g, lc, sums, partial);
    else if (storage == ST_F32) hipLaunchKernelGGL((k_energy_pass<ST_F32, 1>), grid, block, 0, stream, layout, buf, g, lc, sums, partial);
    else hipLaunchKernelGGL((k_energy_pass<ST_F16, 1>), grid, block, 0, stream, layout, buf, g, lc, sums, partial);
    hipLaunchKernelGGL(k_reduce_final_1, dim3(1), dim3(kBlock), 0, stream, partial, (int)blocks, out);
    return hipGetLastError();
}

hipError_t launch_grad_stats(int order, const Geom& g, const double* u, double* partial,
                             double* out, hipStream_t stream)
{
    const unsigned blocks = std::min<unsigned>(kReduceBlocks, grid_for(g.nnodes));
    if (order == 8) hipLaunchKernelGGL(k_grad_stats<8>, dim3(blocks), dim3(kBlock), 0, stream, g, u, partial);
    else hipLaunchKernelGGL(k_grad_stats<2>, dim3(blocks), dim3(kBlock), 0, stream, g, u, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_final_k<8>, dim3(1), dim3(kBlock), 0, stream, partial, (int)blocks, out);
    return hipGetLastError();
}


hipError_t launch_gamma_stats(int storage, int variant, bool exact_gamma, int layout,
                              const void* buf, const Geom& g, const Coll& c,
                              const float* inv_scale, double* partial, double* out,
                              hipStream_t stream)
{
    LoadCtx lc;
    for (int i = 0; i < 27; ++i) lc.inv_scale[i] = inv_scale ? inv_scale[i] : 1.0f;
    const unsigned blocks = std::min<unsigned>(kReduceBlocks, grid_for(g.nnodes));
    GammaFn fn;
    switch (storage) {
    case ST_F64: fn = exact_gamma ? gamma_kernel<ST_F64, true>(variant) : gamma_kernel<ST_F64, false>(variant); break;
    case ST_F32: fn = exact_gamma ? gamma_kernel<ST_F32, true>(variant) : gamma_kernel<ST_F32, false>(variant); break;
    case ST_F32X: fn = exact_gamma ? gamma_kernel<ST_F32X, true>(variant) : gamma_kernel<ST_F32X, false>(variant); break;
    default: fn = exact_gamma ? gamma_kernel<ST_F16, true>(variant) : gamma_kernel<ST_F16, false>(variant); break;
    }
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(kBlock), 0, stream, layout, buf, g, c, lc, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gamma_final, dim3(1), dim3(kBlock), 0, stream, partial, (int)blocks, out);
    return hipGetLastError();
}

int corr_max_nx() { return kCorrMaxN; }
int corr_max_lags() { return kCorrLags * kBlock; }
int corr_blocks(const Geom& g) { return (int)std::min<uint32_t>(kReduceBlocks, g.ny * g.nz); }

hipError_t launch_corr_x(const Geom& g, const double* u, const double* mean_sum, int rmax,
                         double* partial, double* out, hipStream_t stream)
{
    const int blocks = corr_blocks(g);
    hipLaunchKernelGGL(k_corr_x, dim3(blocks), dim3(kBlock), 0, stream, g, u, mean_sum, rmax, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int L2 = 2 * (rmax + 1);
    hipLaunchKernelGGL(k_corr_final, dim3((L2 + kBlock - 1) / kBlock), dim3(kBlock), 0, stream,
                       partial, blocks, rmax, out);
    return hipGetLastError();
}

}  // namespace kbc
