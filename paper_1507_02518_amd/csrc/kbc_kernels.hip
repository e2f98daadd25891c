// kbc_kernels.hip -- gfx950 kernels of the D3Q27 KBC lattice Boltzmann box:
// the fused stream+collide step (pull and AA sweeps), initialisation at the
// product-form equilibrium, layout conversion and FP64 diagnostics.
//
// Streaming follows f_i(x + v_i, t+1) = f'_i(x, t) on a periodic box
// (section I, Eq. Egeneral); the collision is kbc::collide (section IV).
#include <hip/hip_runtime.h>
#include <math.h>

#include "kbc_device.h"
#include "kbc_internal.h"

namespace kbc {

namespace {

constexpr int kBlock = 256;

// Build-time tuning of the step kernel (chosen by measurement).
#ifndef KBC_STEP_BLOCK
#define KBC_STEP_BLOCK 256
#endif
#ifndef KBC_NT_STORE
#define KBC_NT_STORE 1
#endif
#ifndef KBC_WAVES_PER_EU
#define KBC_WAVES_PER_EU 0
#endif
#ifndef KBC_NT_LOAD
#define KBC_NT_LOAD 0
#endif
constexpr int kStepBlock = KBC_STEP_BLOCK;

template <typename T>
__device__ __forceinline__ void st_pop(T* p, T v)
{
    if constexpr (KBC_NT_STORE && sizeof(T) >= 4) __builtin_nontemporal_store(v, p);
    else *p = v;
}

__device__ __forceinline__ uint32_t wrap_add(uint32_t a, int d, uint32_t n)
{
    // a in [0, n), d in {-1, 0, 1}
    if (d > 0) return a + 1 == n ? 0u : a + 1;
    if (d < 0) return a == 0 ? n - 1 : a - 1;
    return a;
}

__device__ __forceinline__ uint32_t node_of(uint32_t x, uint32_t y, uint32_t z, const Geom& g)
{
    return (z * g.ny + y) * g.nx + x;
}

// One node of one step: 27 gathered loads, the collision, 27 stores.
//   pull:    read src[i][x - v_i], write dst[i][x]
//   AA even: read buf[i][x],        write buf[26-i][x]
//   AA odd:  read buf[26-i][x - v_i], write buf[i][x + v_i]
// In both AA sweeps a node reads and writes the same 27 locations, so the
// in-place update is free of races between nodes.
typedef __attribute__((address_space(1))) char gchar_t;

template <int S, int V, int SW, bool GX = false>
__device__ __forceinline__ void node_update(const void* srcv, void* dstv, const Geom& g,
                                            const Coll& c, const int8_t* sexp, uint32_t n)
{
    using T = typename Traits<S>::T;
    using R = typename Traits<S>::R;
    // Addresses are a per-direction plane base (uniform across the wave, kept
    // in scalar registers) plus a 32-bit byte offset within the plane; the
    // host guarantees that a plane is smaller than 4 GiB.
    constexpr uint32_t EB = sizeof(T);
    uint32_t x, y, z;
    node_xyz(n, g, x, y, z);
    const uint32_t rowb = g.row * EB, slabb = g.slab * EB;
    // Pull boxes may be x-blocked (see Geom); AA boxes are always laid out
    // in planes, where the offset of x in its row is x itself.
    auto xoff = [&](uint32_t xx) -> uint32_t {
        if constexpr (SW == SW_PULL) return (xx >> g.xshift) * (g.chunk * EB) + (xx & g.xmask) * EB;
        else return xx * EB;
    };
    const uint32_t xm = x == 0 ? g.nx - 1 : x - 1, xp = x + 1 == g.nx ? 0 : x + 1;
    const uint32_t ym = y == 0 ? g.ny - 1 : y - 1, yp = y + 1 == g.ny ? 0 : y + 1;
    const uint32_t zm = z == 0 ? g.nz - 1 : z - 1, zp = z + 1 == g.nz ? 0 : z + 1;
    // byte offset of coordinate x - v along each axis, indexed by v + 1
    const uint32_t bx[3] = {xoff(xp), xoff(x), xoff(xm)};
    const uint32_t by[3] = {yp * rowb, y * rowb, ym * rowb};
    const uint32_t bz[3] = {zp * slabb, z * slabb, zm * slabb};
    const uint32_t nb = SW == SW_PULL ? bz[1] + by[1] + bx[1] : n * EB;

    // Loads and stores go through two pointers, which in the AA sweeps hold
    // the same buffer; they carry no restrict qualifier, and the order of the
    // accesses comes from the scheduling barrier below.  (One pointer for
    // both measured slower: in the even sweep the compiler stops addressing
    // through scalar plane bases, in the odd FP16 sweep it schedules worse.)
    const char* src = static_cast<const char*>(srcv);
    char* dst = static_cast<char*>(dstv);
    const uint64_t planeb = g.plane * EB;
    // Where every plane is accessed at the same offset (the loads and stores
    // of the even AA sweep, the stores of the pull sweep) the compiler would
    // fold buffer + offset into one 64-bit vector address and add each
    // plane's distance with 64-bit vector arithmetic, two VALU instructions
    // per access.  Hiding the plane base (a scalar) keeps the scalar-base +
    // 32-bit-offset form, as for the shifted accesses.  The base passes
    // through a global-address-space pointer so that the compiler still
    // knows the accesses are global rather than flat.
    auto plane = [&](auto* b, int slot, bool hide) {
        auto* p = b + slot * planeb;
        if (hide) {
            gchar_t* q = (gchar_t*)p;
            asm volatile("" : "+s"(q));
            p = (decltype(p))q;
        }
        return p;
    };
    auto ld = [&](int slot, uint32_t off) -> T {
        const T* p = reinterpret_cast<const T*>(plane(src, slot, SW == SW_AA_EVEN) + off);
        if constexpr (KBC_NT_LOAD) return __builtin_nontemporal_load(p);
        else return *p;
    };
    auto st = [&](int slot, uint32_t off, T v) {
        st_pop(reinterpret_cast<T*>(plane(dst, slot, SW != SW_AA_ODD) + off), v);
    };

    // FP16 scale exponent of direction i: the host makes it equal for i and
    // its opposite, so 14 distinct values (scalar registers) serve all 27
    auto ex = [&](int i) -> int { return sexp[i <= 13 ? i : 26 - i]; };

    R f[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        const int ax = i % 3, ay = (i / 3) % 3, az = i / 9;
        if constexpr (SW == SW_PULL) {
            f[i] = decode_exp<S>(ld(i, bz[az] + by[ay] + bx[ax]), ex(i));
        } else if constexpr (SW == SW_AA_EVEN) {
            f[i] = decode_exp<S>(ld(i, nb), ex(i));
        } else {
            f[i] = decode_exp<S>(ld(opp(i), bz[az] + by[ay] + bx[ax]), ex(i));
        }
    }

    if constexpr (SW != SW_PULL) {
        // AA sweeps read and write the same 27 locations through src and
        // dst (one buffer): the instruction scheduler may not move any
        // instruction across this point, so every load is issued before any
        // store (checked on the built code by the test suite)
        __builtin_amdgcn_sched_barrier(0);
    }

    collide<S, V, GX>(f, c);

    // AA odd sweep: store offsets x + v are formed after the collision, from
    // the coordinates alone, so they do not occupy registers across it (the
    // empty asm only hides the coordinates from common-subexpression reuse)
    uint32_t fx[3] = {0, 0, 0}, fy[3] = {0, 0, 0}, fz[3] = {0, 0, 0};
    if constexpr (SW == SW_AA_ODD) {
        uint32_t x2 = x, y2 = y, z2 = z;
        asm volatile("" : "+v"(x2), "+v"(y2), "+v"(z2));
        fx[0] = xoff(x2 == 0 ? g.nx - 1 : x2 - 1);
        fx[1] = xoff(x2);
        fx[2] = xoff(x2 + 1 == g.nx ? 0 : x2 + 1);
        fy[0] = (y2 == 0 ? g.ny - 1 : y2 - 1) * rowb;
        fy[1] = y2 * rowb;
        fy[2] = (y2 + 1 == g.ny ? 0 : y2 + 1) * rowb;
        fz[0] = (z2 == 0 ? g.nz - 1 : z2 - 1) * slabb;
        fz[1] = z2 * slabb;
        fz[2] = (z2 + 1 == g.nz ? 0 : z2 + 1) * slabb;
    }

#pragma unroll
    for (int i = 0; i < 27; ++i) {
        const int ax = i % 3, ay = (i / 3) % 3, az = i / 9;
        if constexpr (SW == SW_PULL) {
            st(i, nb, encode_exp<S>(f[i], ex(i)));
        } else if constexpr (SW == SW_AA_EVEN) {
            st(opp(i), nb, encode_exp<S>(f[i], ex(i)));
        } else {
            st(i, fz[az] + fy[ay] + fx[ax], encode_exp<S>(f[i], ex(i)));
        }
    }
}

// Fused step of one box: one thread per node, workgroups of up to
// kStepBlock threads (the launch picks the size).  GX: exact stabilizer.
template <int S, int V, int SW, bool GX>
__global__ void __launch_bounds__(kStepBlock)
#if KBC_WAVES_PER_EU
__attribute__((amdgpu_waves_per_eu(KBC_WAVES_PER_EU, 8)))
#endif
k_step(StepParams p)
{
    const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= p.g.nnodes) return;
    node_update<S, V, SW, GX>(p.src, p.dst, p.g, p.c, p.scale_exp, n);
}

typedef __attribute__((address_space(1))) char gchar;

// Batched step over one launch group of a pool's boxes (AA sweep SW, in
// place).  A tile is `sub` consecutive block-sized runs of one box's nodes.
// Each block takes tiles blockIdx.x, blockIdx.x + gridDim.x, ...; a tile
// belongs to the last box whose first tile is not after it (binary search
// over the compact array of first tiles).  Boxes are disjoint in memory and
// each node is updated by exactly one thread, so a box evolves exactly as it
// would alone.
template <int S, int V, int SW>
__global__ void __launch_bounds__(kPoolMaxBlock) k_pool_step(const PoolBox* __restrict__ table,
                                                             const uint32_t* __restrict__ ttable,
                                                             const PoolMeta* __restrict__ meta,
                                                             int k)
{
    const PoolBox* __restrict__ boxes = table + meta->first;
    const uint32_t* __restrict__ tstart = ttable + meta->first;
    const uint32_t n_tiles = meta->n_tiles;
    const uint32_t n_active = meta->n_active;
    const uint32_t block = meta->block;
    const uint32_t sub = meta->sub;
#pragma unroll 1
    for (uint32_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        uint32_t lo = 0, hi = n_active;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (tstart[mid] <= tile) lo = mid;
            else hi = mid;
        }
        const PoolBox& b = boxes[lo];
        if (k >= b.steps) continue;
        // FP16: the box's scale exponents, staged in LDS once per tile so the
        // node update reads them there rather than from the box table
        __shared__ int8_t s_exp[28];
        if constexpr (S == ST_F16) {
            __syncthreads();
            if (threadIdx.x < 28) s_exp[threadIdx.x] = b.scale_exp[threadIdx.x];
            __syncthreads();
        }
        // the box's constants as values, so the population stores cannot be
        // taken to alias them
        const Geom g = b.g;
        const Coll c = b.c;
        // the table holds a generic pointer; it addresses global memory, and
        // saying so lets the compiler use global (not flat) loads and stores
        gchar* const gbuf = (gchar*)b.buf;
        const uint32_t first = (tile - tstart[lo]) * sub * block;
#pragma unroll 1
        for (uint32_t r = 0; r < sub; ++r) {
            const uint32_t n = first + r * block + threadIdx.x;
            if (n < g.nnodes) {
                // loads and stores see the buffer through two global pointers,
                // as in the single-box kernel (they are kept apart by the
                // scheduling barrier in node_update)
                gchar* sbuf = gbuf;
                gchar* dbuf = gbuf;
                asm volatile("" : "+s"(sbuf));
                asm volatile("" : "+s"(dbuf));
                node_update<S, V, SW>((void*)sbuf, (void*)dbuf, g, c, s_exp, n);
            }
        }
    }
}

using PoolFn = void (*)(const PoolBox*, const uint32_t*, const PoolMeta*, int);

template <int S, int V>
PoolFn pool_fn_sw(int sw)
{
    return sw == SW_AA_EVEN ? k_pool_step<S, V, SW_AA_EVEN> : k_pool_step<S, V, SW_AA_ODD>;
}

template <int S>
PoolFn pool_fn_v(int v, int sw)
{
    switch (v) {
    case V_D: return pool_fn_sw<S, V_D>(sw);
    case V_DT: return pool_fn_sw<S, V_DT>(sw);
    case V_DQ: return pool_fn_sw<S, V_DQ>(sw);
    case V_CD: return pool_fn_sw<S, V_CD>(sw);
    case V_CDT: return pool_fn_sw<S, V_CDT>(sw);
    case V_CDQ: return pool_fn_sw<S, V_CDQ>(sw);
    case V_CDTQ: return pool_fn_sw<S, V_CDTQ>(sw);
    default: return pool_fn_sw<S, V_DTQ>(sw);
    }
}

using StepFn = void (*)(StepParams);

template <int S, int V, bool GX>
constexpr StepFn step_fn(int sw)
{
    return sw == SW_PULL ? k_step<S, V, SW_PULL, GX>
                         : (sw == SW_AA_EVEN ? k_step<S, V, SW_AA_EVEN, GX>
                                             : k_step<S, V, SW_AA_ODD, GX>);
}

template <int S, bool GX>
StepFn step_fn_v(int v, int sw)
{
    switch (v) {
    case V_D: return step_fn<S, V_D, GX>(sw);
    case V_DT: return step_fn<S, V_DT, GX>(sw);
    case V_DQ: return step_fn<S, V_DQ, GX>(sw);
    case V_CD: return step_fn<S, V_CD, GX>(sw);
    case V_CDT: return step_fn<S, V_CDT, GX>(sw);
    case V_CDQ: return step_fn<S, V_CDQ, GX>(sw);
    case V_CDTQ: return step_fn<S, V_CDTQ, GX>(sw);
    default: return step_fn<S, V_DTQ, GX>(sw);
    }
}

template <bool GX>
StepFn step_fn_sv(int storage, int v, int sw)
{
    switch (storage) {
    case ST_F64: return step_fn_v<ST_F64, GX>(v, sw);
    case ST_F32: return step_fn_v<ST_F32, GX>(v, sw);
    case ST_F32X: return step_fn_v<ST_F32X, GX>(v, sw);
    default: return step_fn_v<ST_F16, GX>(v, sw);
    }
}

// ---------------------------------------------------------------------------
// Storage location of canonical F_i(x) in a layout: the slot and the element
// index in the buffer.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t locate(int layout, int i, uint32_t x, uint32_t y, uint32_t z,
                                           const Geom& g, int& slot)
{
    const int vx = vel(i, 0), vy = vel(i, 1), vz = vel(i, 2);
    if (layout == LY_AA_EVEN) {
        slot = i;
        return pop_index(g, slot, x, y, z);
    }
    // the pull sweep reads F_i(x) from the post-collision buffer at x - v_i;
    // the odd AA sweep from the opposite slot there
    slot = layout == LY_PULL ? i : opp(i);
    return pop_index(g, slot, wrap_add(x, -vx, g.nx), wrap_add(y, -vy, g.ny),
                     wrap_add(z, -vz, g.nz));
}

template <int S>
__device__ __forceinline__ double load_full(const void* buf, uint64_t idx, int slot, int i,
                                            const float* inv_scale)
{
    using T = typename Traits<S>::T;
    const T v = static_cast<const T*>(buf)[idx];
    if constexpr (S == ST_F64) return (double)v;
    else if constexpr (S == ST_F32) return weight(i) + (double)v;
    else return weight(i) + (double)((float)v * inv_scale[slot]);
}

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

struct LoadCtx {
    float inv_scale[27];
};

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

// rho = sum_i f_i, rho u = sum_i v_i f_i (section I), in FP64.  Deviation
// forms sum the stored deviations and add the weights' share (1, 0).
template <int S>
__global__ void __launch_bounds__(kBlock) k_moments(int layout, const void* buf, Geom g, LoadCtx lc,
                                                    double* __restrict__ rho,
                                                    double* __restrict__ u, int* flag)
{
    const uint32_t n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.nnodes) return;
    uint32_t x, y, z;
    node_xyz(n, g, x, y, z);
    double m = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
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
    const double ux = jx * ir, uy = jy * ir, uz = jz * ir;
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

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int K>
__device__ __forceinline__ void block_sum(double (&acc)[K], double* out)
{
    __shared__ double red[kBlock / 64][K];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = wave_sum(acc[k]);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) red[wave][k] = acc[k];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double s = 0.0;
            for (int w = 0; w < kBlock / 64; ++w) s += red[w][k];
            out[k] = s;
        }
}

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

// Per-block sums of gamma and gamma^2 and the block's min and max of the
// stabilizer that the next step would use at each node (the collision up to
// step 6 on the stored state; nothing is written back).
template <int S, int V, bool GX>
__global__ void __launch_bounds__(kBlock) k_gamma_stats(int layout, const void* buf, Geom g, Coll c,
                                                        LoadCtx lc, double* __restrict__ partial)
{
    using T = typename Traits<S>::T;
    using R = typename Traits<S>::R;
    double sum = 0.0, sum2 = 0.0, lo = __builtin_inf(), hi = -__builtin_inf();
    for (uint32_t n = blockIdx.x * kBlock + threadIdx.x; n < g.nnodes; n += gridDim.x * kBlock) {
        uint32_t x, y, z;
        node_xyz(n, g, x, y, z);
        R f[27];
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            int slot;
            const uint64_t idx = locate(layout, i, x, y, z, g, slot);
            f[i] = decode<S>(static_cast<const T*>(buf)[idx], lc.inv_scale[slot]);
        }
        double gam = 0.0;
        collide<S, V, GX>(f, c, &gam);
        sum += gam;
        sum2 += gam * gam;
        lo = fmin(lo, gam);
        hi = fmax(hi, gam);
    }
    double acc[2] = {sum, sum2};
    block_sum<2>(acc, partial + 4 * blockIdx.x);
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
        // the block sums went to partial[4b], [4b+1]; min and max follow
        partial[4 * blockIdx.x + 2] = lo;
        partial[4 * blockIdx.x + 3] = hi;
    }
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

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_step(int storage, int variant, int sweep, bool exact_gamma, const StepParams& p,
                       hipStream_t stream)
{
    // the AA kernels address populations in planes (see node_update)
    if (sweep != SW_PULL && !geom_is_planes(p.g)) return hipErrorInvalidValue;
    const StepFn fn = exact_gamma ? step_fn_sv<true>(storage, variant, sweep)
                                  : step_fn_sv<false>(storage, variant, sweep);
    // One wavefront per workgroup for the exact stabilizer (one wave per
    // SIMD: 64-thread workgroups fill the CUs more evenly; at 256^3 the pull
    // sweep ran 14% (FP64) and 5% (FP32-X) faster than with 256 threads, the
    // AA sweeps 12% and 8%), kStepBlock threads otherwise (64 measured within
    // +-2% for the other pull forms, 5% slower for FP16 pull, and 17-33%
    // slower for the AA sweeps).
    const uint32_t block = exact_gamma ? 64u : (uint32_t)kStepBlock;
    hipLaunchKernelGGL(fn, dim3((p.g.nnodes + block - 1) / block), dim3(block), 0, stream, p);
    return hipGetLastError();
}

hipError_t launch_pool_step(int storage, int variant, int sweep, const PoolBox* boxes,
                            const uint32_t* tstart, const PoolMeta* meta, int k, int block,
                            int grid, hipStream_t stream)
{
    if (block < 64 || block > kPoolMaxBlock || block % 64 || grid < 1) return hipErrorInvalidValue;
    if (sweep != SW_AA_EVEN && sweep != SW_AA_ODD) return hipErrorInvalidValue;
    PoolFn fn;
    switch (storage) {
    case ST_F64: fn = pool_fn_v<ST_F64>(variant, sweep); break;
    case ST_F32: fn = pool_fn_v<ST_F32>(variant, sweep); break;
    case ST_F32X: fn = pool_fn_v<ST_F32X>(variant, sweep); break;
    default: fn = pool_fn_v<ST_F16>(variant, sweep); break;
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

namespace {
using GammaFn = void (*)(int, const void*, Geom, Coll, LoadCtx, double*);

template <int S, bool GX>
GammaFn gamma_fn_v(int v)
{
    switch (v) {
    case V_D: return k_gamma_stats<S, V_D, GX>;
    case V_DT: return k_gamma_stats<S, V_DT, GX>;
    case V_DQ: return k_gamma_stats<S, V_DQ, GX>;
    case V_CD: return k_gamma_stats<S, V_CD, GX>;
    case V_CDT: return k_gamma_stats<S, V_CDT, GX>;
    case V_CDQ: return k_gamma_stats<S, V_CDQ, GX>;
    case V_CDTQ: return k_gamma_stats<S, V_CDTQ, GX>;
    default: return k_gamma_stats<S, V_DTQ, GX>;
    }
}

template <bool GX>
GammaFn gamma_fn(int storage, int v)
{
    switch (storage) {
    case ST_F64: return gamma_fn_v<ST_F64, GX>(v);
    case ST_F32: return gamma_fn_v<ST_F32, GX>(v);
    case ST_F32X: return gamma_fn_v<ST_F32X, GX>(v);
    default: return gamma_fn_v<ST_F16, GX>(v);
    }
}
}  // namespace

hipError_t launch_gamma_stats(int storage, int variant, bool exact_gamma, int layout,
                              const void* buf, const Geom& g, const Coll& c,
                              const float* inv_scale, double* partial, double* out,
                              hipStream_t stream)
{
    LoadCtx lc;
    for (int i = 0; i < 27; ++i) lc.inv_scale[i] = inv_scale ? inv_scale[i] : 1.0f;
    const unsigned blocks = std::min<unsigned>(kReduceBlocks, grid_for(g.nnodes));
    const GammaFn fn = exact_gamma ? gamma_fn<true>(storage, variant) : gamma_fn<false>(storage, variant);
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
