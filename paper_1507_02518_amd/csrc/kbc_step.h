// kbc_step.h -- device code of the fused stream+collide step shared by the
// translation units that instantiate it (kbc_step_inst.hip, one per storage
// form and stabilizer mode) and by kbc_kernels.hip (index helpers and the
// deterministic block reduction).
//
// Streaming follows f_i(x + v_i, t+1) = f'_i(x, t) on a periodic box
// (section I, Eq. Egeneral); the collision is kbc::collide (section IV).
#pragma once

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
#ifndef KBC_AA_ALIGNED
#define KBC_AA_ALIGNED 1
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

// ALN (AA odd sweep of a single box, FP64 and FP32-X storage): line-aligned
// stores.  The value that
// node x sends to x + v_i is stored by the thread of node x + v_x of the
// same row (its own x, so each store instruction of a wave covers whole cache
// lines); the values cross between threads through LDS after the collision.
// Where that thread is not in the workgroup (a row split between
// workgroups) the owner stores its value itself, as without ALN.  n0: first
// node of the workgroup's contiguous range of blockDim.x nodes; `store`:
// whether this thread's node is real (a thread past the last node takes the
// last node's inputs, so its LDS entries are defined, and stores nothing).
//
// C64 (pull sweep of a box x-blocked in chunks of 64 nodes): the chunk
// geometry is a compile-time constant, so the 27 directions of a chunk lie
// at fixed byte distances that the loads and stores carry in their
// immediate offset field where it reaches (FP16: all 27, 128 bytes apart)
// instead of one scalar base per direction.
template <int S, int V, int SW, bool GX = false, bool ALN = false, bool C64 = false>
__device__ __forceinline__ void node_update(const void* srcv, void* dstv, const Geom& g,
                                            const Coll& c, const int8_t* sexp, uint32_t n,
                                            uint32_t n0 = 0, bool store = true)
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
        if constexpr (C64) return (xx >> 6) * (27 * 64 * EB) + (xx & 63) * EB;
        else if constexpr (SW == SW_PULL) return (xx >> g.xshift) * (g.chunk * EB) + (xx & g.xmask) * EB;
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
    const uint64_t planeb = C64 ? 64 * EB : g.plane * EB;
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

    if constexpr (ALN) {
        static_assert(SW == SW_AA_ODD, "aligned stores are for the odd AA sweep");
        // the 18 directions with v_x != 0 cross lanes: slot k = 2 (i / 3) +
        // (v_x > 0)
        // The relaxed populations are pinned here, before any branch: the
        // conditional stores below would otherwise let the compiler sink the
        // last operations of the relaxation into them, where they no longer
        // fuse as in the other sweeps and the pool kernel (a last-bit
        // difference between a box alone and in the pool).
#pragma unroll
        for (int i = 0; i < 27; ++i) asm volatile("" : "+v"(f[i]));
        __shared__ T xch[18][kStepBlock];
        const uint32_t t = threadIdx.x, nb_ = blockDim.x;
        // directions with v_x = 0 stay in their lane and are stored at once
        // (a location is read only by the node that writes it, which has
        // loaded its inputs already); the others go through LDS, so no
        // population stays in a register across the barrier
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            const int ay = (i / 3) % 3, az = i / 9;
            if (i % 3 == 1) {
                if (store) st(i, fz[az] + fy[ay] + fx[1], encode_exp<S>(f[i], ex(i)));
            } else {
                xch[2 * (i / 3) + (i % 3 == 2)][t] = encode_exp<S>(f[i], ex(i));
            }
        }
        __syncthreads();
        // node index of (0, y, z) relative to the workgroup's first node;
        // unsigned arithmetic: a node outside [n0, n0 + blockDim) maps to an
        // index >= blockDim
        const uint32_t row0 = n - x - n0;
        const uint32_t xl = x == 0 ? g.nx - 1 : x - 1, xr = x + 1 == g.nx ? 0 : x + 1;
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            const int ax = i % 3, ay = (i / 3) % 3, az = i / 9;
            if (ax == 1) continue;
            const int k = 2 * (i / 3) + (ax == 2);
            // the value that lands on this x comes from x - v_x; this node's
            // own value goes to x + v_x
            const uint32_t src = row0 + (ax == 2 ? xl : xr);
            const uint32_t dst = row0 + (ax == 2 ? xr : xl);
            if (store && src < nb_) st(i, fz[az] + fy[ay] + fx[1], xch[k][src]);
            if (store && dst >= nb_) st(i, fz[az] + fy[ay] + fx[ax], xch[k][t]);
        }
    } else {
        // the stores at the node's own offset: a copy the compiler cannot
        // tie to the loads' 64-bit address arithmetic keeps every store in
        // the scalar-base + 32-bit-offset form (without it each store takes a
        // 64-bit vector add, 27 VALU instructions per node)
        uint32_t nbs = nb;
        if constexpr (SW != SW_AA_ODD) asm volatile("" : "+v"(nbs));
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            const int ax = i % 3, ay = (i / 3) % 3, az = i / 9;
            if constexpr (SW == SW_PULL) {
                st(i, nbs, encode_exp<S>(f[i], ex(i)));
            } else if constexpr (SW == SW_AA_EVEN) {
                st(opp(i), nbs, encode_exp<S>(f[i], ex(i)));
            } else {
                st(i, fz[az] + fy[ay] + fx[ax], encode_exp<S>(f[i], ex(i)));
            }
        }
    }
}

// Workgroup b of a launch runs on XCD b mod 8 (the dispatcher deals
// workgroups to the eight XCDs in turn).  ORDER_PLAIN keeps that: the XCDs
// advance through the box side by side, one front, and consecutive
// workgroups sit in different L2 caches.  The AA sweeps take one of two
// other orders, chosen by the host per box:
//   ORDER_PAIRS: XCD x's k-th workgroup takes block 2 (8 (k / 2) + x) +
//   k % 2, still one front, but each XCD takes two consecutive blocks, so
//   the two halves of a 512-node row (read shifted by one node in x by the
//   odd sweep) meet in one L2.  FP16 AA at 512^3 2.7-5.4% and FP32 AA 1-3.6%
//   faster than the plain order.  Taken only where a row is longer than a
//   workgroup: on shorter rows nothing is split, and boxes of 128^3 (in the
//   last-level cache) ran 15-21% slower in pairs (FP32-X, FP16).
//   ORDER_EIGHTHS: each XCD takes one contiguous eighth of the blocks (XCD
//   j's k-th workgroup gets block start(j) + k), eight fronts, each reading
//   the z - 1 and z + 1 slabs of its own nodes.  Taken where the three
//   slabs an AA sweep reads at once, over all 27 planes, exceed half of the
//   256 MB last-level cache (FP64 at 512^3: 170 MB, 7-9% faster per sweep
//   pair); on smaller slabs one front measured faster (FP64 AA at 256^3 9%,
//   FP32 and FP16 AA at 512^3 0-2%).
// The pull sweep (FP64 at 512^3 the same in either order) and the exact
// stabilizer (ALU-bound, one-wave workgroups) keep the plain order.  Blocks
// past the last whole group of 16 (pairs) or at the tail (eighths) keep
// their index in the pairs order and are spread in the eighths order.
__device__ __forceinline__ uint32_t step_block(uint32_t b, uint32_t grid, uint32_t order)
{
    if (order == ORDER_PAIRS) {
        const uint32_t full = grid & ~15u;
        if (b >= full) return b;
        const uint32_t x = b & 7u, k = b >> 3;
        return ((k >> 1) * 8u + x) * 2u + (k & 1u);
    }
    if (order == ORDER_EIGHTHS) {
        const uint32_t j = b & 7u, k = b >> 3, q = grid >> 3, r = grid & 7u;
        return j * q + (j < r ? j : r) + k;
    }
    return b;
}

// Fused step of one box: one thread per node, workgroups of up to
// kStepBlock threads (the launch picks the size).  GX: exact stabilizer.
// C64: pull sweep on 64-node chunks (node_update).
#ifndef KBC_GX_WAVES_PER_EU
#define KBC_GX_WAVES_PER_EU 1
#endif
template <int S, int V, int SW, bool GX, bool C64 = false>
__global__ void __launch_bounds__(kStepBlock)
#if KBC_WAVES_PER_EU
__attribute__((amdgpu_waves_per_eu(KBC_WAVES_PER_EU, 8)))
#else
__attribute__((amdgpu_waves_per_eu(GX ? KBC_GX_WAVES_PER_EU : 1, 8)))
#endif
k_step(StepParams p)
{
    // pairs only where a row is longer than a workgroup: the halves of a
    // split row are what that order keeps in one L2
    uint32_t order = SW != SW_PULL && !GX ? p.xcd_order : ORDER_PLAIN;
    if (order == ORDER_PAIRS && p.g.nx <= blockDim.x) order = ORDER_PLAIN;
    const uint32_t n0 = step_block(blockIdx.x, gridDim.x, order) * blockDim.x;
    const uint32_t n = n0 + threadIdx.x;
    // aligned stores where the exchange costs no occupancy: FP64 (2 waves
    // per SIMD either way) and FP32 with the FP64-formed non-equilibrium (3);
    // the plain FP32 and FP16 sweeps would drop from 4 waves to 3 (FP32 at
    // 512^3 measured 5% slower with the exchange)
    if constexpr (SW == SW_AA_ODD && !GX && KBC_AA_ALIGNED && (S == ST_F64 || S == ST_F32X)) {
        // every thread reaches the workgroup barrier of the aligned stores
        const bool real = n < p.g.nnodes;
        node_update<S, V, SW, GX, true>(p.src, p.dst, p.g, p.c, p.scale_exp,
                                        real ? n : p.g.nnodes - 1, n0, real);
    } else {
        if (n >= p.g.nnodes) return;
        node_update<S, V, SW, GX, false, C64>(p.src, p.dst, p.g, p.c, p.scale_exp, n);
    }
}

typedef __attribute__((address_space(1))) char gchar;

// Batched step over one launch group of a pool's boxes (AA sweep SW, in
// place).  A tile is `sub` consecutive block-sized runs of one box's nodes.
// Each block takes tiles blockIdx.x, blockIdx.x + gridDim.x, ...; a tile
// belongs to the last box whose first tile is not after it (binary search
// over the compact array of first tiles).  Boxes are disjoint in memory and
// each node is updated by exactly one thread, so a box evolves exactly as it
// would alone.  ONE: the launch has a block for every tile and sub = 1, so a
// block takes exactly one run of nodes; without the two loops the kernel
// keeps no loop state in scalar registers (the FP32-X odd sweep spilled 27
// of them to vector lanes) and runs one large box as fast as the single-box
// kernel.
template <int S, int V, int SW, bool ONE = false>
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
    const uint32_t sub = ONE ? 1u : meta->sub;
    // one tile; false when its box has no step to take in this launch
    auto run_tile = [&](uint32_t tile) {
        uint32_t lo = 0, hi = n_active;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (tstart[mid] <= tile) lo = mid;
            else hi = mid;
        }
        const PoolBox& b = boxes[lo];
        if (k >= b.steps) return;
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
        auto run = [&](uint32_t r) {
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
        };
        if constexpr (ONE) {
            run(0);
        } else {
#pragma unroll 1
            for (uint32_t r = 0; r < sub; ++r) run(r);
        }
    };
    if constexpr (ONE) {
        if (blockIdx.x < n_tiles) run_tile(blockIdx.x);
    } else {
#pragma unroll 1
        for (uint32_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) run_tile(tile);
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
// Deterministic FP64 block reduction: butterfly within the wavefront, fixed
// order across wavefronts.
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

// Per-block sums of gamma and gamma^2 and the block's min and max of the
// stabilizer that the next step would use at each node (the collision on the
// stored state as far as gamma; nothing is written back).
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
}  // namespace

}  // namespace kbc
