// kbc_internal.h -- host-side interface between the C-ABI layer and the
// kernel launchers (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kbc_device.h"

namespace kbc {

// Population storage layout of one box (all modes are [27][nz][ny][nx]):
//   pull:  buffer `cur` holds the post-collision P(t-1) so that
//          F_i(x, t) = cur[i][x - v_i] (at t = 0, cur[i][x] = f^eq_i(x + v_i));
//   AA:    even t: F_i(x, t) = buf[i][x]; odd t: F_i(x, t) = buf[26-i][x - v_i].
enum Layout : int { LY_PULL = 0, LY_AA_EVEN = 1, LY_AA_ODD = 2 };

// Population layouts of a box (see Geom).  Planes [27][nz][ny][nx], each
// followed by `pad` unused elements:
inline void geom_planes(Geom& g, uint64_t pad)
{
    g.plane = (uint64_t)g.nnodes + pad;
    g.row = g.nx;
    g.slab = g.nx * g.ny;
    g.chunk = 0;
    g.xshift = 31;
    g.xmask = 0x7fffffffu;
}

// x-blocked [nz][ny][nx/B][27][B]: the 27 populations of B nodes adjacent in
// x lie in one contiguous run, B = 64 or 32 where it divides nx, else B = nx.
inline void geom_blocked(Geom& g)
{
    const uint32_t b = g.nx % 64 == 0 ? 64 : (g.nx % 32 == 0 ? 32 : g.nx);
    g.plane = b;
    g.row = 27 * g.nx;
    g.slab = 27 * g.nx * g.ny;
    if (b == g.nx) {
        g.chunk = 0;
        g.xshift = 31;
        g.xmask = 0x7fffffffu;
    } else {
        g.chunk = 27 * b;
        g.xshift = b == 64 ? 6 : 5;
        g.xmask = b - 1;
    }
}

inline bool geom_is_planes(const Geom& g) { return g.row == g.nx && g.xshift == 31 && g.plane >= g.nnodes; }

// Elements of the buffer that the layout spans.
inline uint64_t geom_extent(const Geom& g) { return pop_index(g, 26, g.nx - 1, g.ny - 1, g.nz - 1) + 1; }

// Bytes spanned by the populations of one slot (the 32-bit offsets of the
// step kernels address within this span from the slot's base).
inline uint64_t geom_slot_span_bytes(const Geom& g, size_t elem)
{
    return (pop_index(g, 0, g.nx - 1, g.ny - 1, g.nz - 1) + 1) * elem;
}

// Record the message returned by kbc_last_error() on this thread.
void set_last_error(const char* msg);

// One time step of one box (src -> dst for pull; in place for AA).
hipError_t launch_step(int storage, int variant, int sweep, bool exact_gamma, const StepParams& p,
                       hipStream_t stream);

// The kernel and launch shape launch_step uses (for building graphs of steps).
using StepFn = void (*)(StepParams);
hipError_t step_launch_shape(int storage, int variant, int sweep, bool exact_gamma, const Geom& g,
                             StepFn* fn, uint32_t* grid, uint32_t* block);

// Write f^eq(rho, u) of device fields u [3][N], rho [N] (may be NULL) into the
// storage buffer in the given layout.
hipError_t launch_init_feq(int storage, int layout, void* buf, const Geom& g,
                           const float* scale, const double* u, const double* rho,
                           hipStream_t stream);

// Validity of an initial state: sets *flag (device int, pre-zeroed) to 1 if
// some |u_a| >= 1 or rho <= 0 or a value is not finite.
hipError_t launch_check_init(const Geom& g, const double* u, const double* rho, int* flag,
                             hipStream_t stream);

// Per-direction max |f^eq_i - W_i| over the box (device float[27], zeroed
// by the callee) for choosing FP16 scales.
hipError_t launch_feq_dev_max(const Geom& g, const double* u, const double* rho,
                              unsigned* max_bits, hipStream_t stream);

// Per-direction max |f_i - W_i| of a canonical FP64 population field.
hipError_t launch_pop_dev_max(const Geom& g, const double* f, unsigned* max_bits,
                              hipStream_t stream);

// Canonical F(t) [27][N] FP64 <-> storage in the given layout.
hipError_t launch_gather_pop(int storage, int layout, const void* buf, const Geom& g,
                             const float* inv_scale, double* f, hipStream_t stream);
hipError_t launch_scatter_pop(int storage, int layout, void* buf, const Geom& g,
                              const float* scale, const double* f, hipStream_t stream);

// F(t) at selected nodes: out [count][27] FP64, nodes [count] (in range).
hipError_t launch_sample_pop(int storage, int layout, const void* buf, const Geom& g,
                             const float* inv_scale, const uint32_t* nodes, int count,
                             double* out, hipStream_t stream);

// rho [N] (nullable) and u [3][N] of F(t); sets *flag if a value is not finite.
hipError_t launch_moments(int storage, int layout, const void* buf, const Geom& g,
                          const float* inv_scale, double* rho, double* u, int* flag,
                          hipStream_t stream);

// Plain streaming copy of n16 16-byte words.
hipError_t launch_copy16(void* dst, const void* src, size_t n16, hipStream_t stream);
hipError_t launch_rewrite16(void* p, size_t n16, hipStream_t stream);

// Deterministic FP64 reductions over a velocity field u [3][N].
//   kind 0: out[0..2] = sum_x u_a(x)
//   kind 1: out[0]    = sum_x |u(x) - mean|^2     (mean = in[0..2] / N)
//   kind 2: out[0]    = sum_x |curl_FD2 u(x)|^2
// Flow statistics.  grad: out[8] = sums over nodes of |curl u|^2,
// sum_ab (d_a u_b + d_b u_a)^2, (div u)^2, (du_x/dx)^n for n = 2..6, with the
// central stencil of the given order (2 or 8); partial: reduce_partials() * 8.
hipError_t launch_grad_stats(int order, const Geom& g, const double* u, double* partial,
                             double* out, hipStream_t stream);
// gamma of the next collision at every node: out[4] = sum, sum of squares,
// min, max; partial: reduce_partials() * 4.
hipError_t launch_gamma_stats(int storage, int variant, bool exact_gamma, int layout,
                              const void* buf, const Geom& g, const Coll& c,
                              const float* inv_scale, double* partial, double* out,
                              hipStream_t stream);
// x-correlation sums: out[2r + c] = sum over nodes of u'_c(x) u'_c(x + r),
// c = 0 (x component), 1 (y component), r = 0..rmax; requires
// nx <= corr_max_nx(), rmax < corr_max_lags(); partial: corr_blocks(g) *
// 2 (rmax + 1) doubles; mean_sum: the three sums of u.
int corr_max_nx();
int corr_max_lags();
int corr_blocks(const Geom& g);
hipError_t launch_corr_x(const Geom& g, const double* u, const double* mean_sum, int rmax,
                         double* partial, double* out, hipStream_t stream);

// Kinetic-energy sum of F(t) read straight from the populations (no velocity
// field in memory): *out = sum_x |u(x) - mean|^2, the same bits as
// launch_moments + launch_reduce kinds 0 and 1.  partial: reduce_partials() * 3
// doubles; sums: 3 doubles (left holding the sums of u).
hipError_t launch_energy_direct(int storage, int layout, const void* buf, const Geom& g,
                                const float* inv_scale, double* partial, double* sums,
                                double* out, hipStream_t stream);

// `partial` is device scratch of reduce_partials() doubles * 3.
int reduce_partials();
hipError_t launch_reduce(int kind, const Geom& g, const double* u, const double* mean_sum,
                         double* partial, double* out, hipStream_t stream);

// ---------------------------------------------------------------------------
// Batched ensemble (pool): many independent AA boxes advanced by one launch.
// ---------------------------------------------------------------------------
struct PoolBox {
    void* buf;            // the box's population array (AA layout, in place)
    Geom g;
    Coll c;
    uint32_t tile0;       // first tile of the box in the current batch
    uint32_t ntiles;      // ceil(nnodes / (block * sub))
    int32_t parity0;      // t mod 2 at the start of the batch
    int32_t steps;        // steps the box takes in the current batch
    int8_t scale_exp[28]; // FP16 storage: stored = (f - W) * 2^scale_exp[i]
};

// One launch group of a batch: boxes[first .. first + n_active) of the
// batch's box table, all at the same parity, sorted by tile0 (tiles are
// numbered from 0 within the group).
struct PoolMeta {
    uint32_t first;       // index of the group's first box in the table
    uint32_t n_active;    // boxes in the group
    uint32_t n_tiles;     // tiles in the group
    uint32_t block;       // threads per block
    uint32_t sub;         // block-sized sub-tiles per tile
};

constexpr int kPoolMaxBlock = 512;

// Step k (0-based) of a batch for one launch group: every box of the group
// with k < steps applies the AA sweep `sweep` (SW_AA_EVEN or SW_AA_ODD).
// Persistent grid-stride loop over the group's tiles; block <= 512.
// boxes and tstart are the whole table (tstart[b] = boxes[b].tile0, a
// compact copy for the tile -> box search); meta is the group's entry.
// one: the launch has a block for every tile of the group and one run of
// nodes per tile (sub = 1), so the single-tile kernel applies
hipError_t launch_pool_step(int storage, int variant, int sweep, const PoolBox* boxes,
                            const uint32_t* tstart, const PoolMeta* meta, int k, int block,
                            int grid, bool one, hipStream_t stream);

// ---------------------------------------------------------------------------
// Kernel tables.  The step, pool and stabilizer-statistics kernels are
// instantiated in kbc_step_inst.hip, once per storage form S and stabilizer
// mode GX (exact root or estimate), so that the eight instances compile in
// parallel; these functions return the kernel for a variant and sweep.
// ---------------------------------------------------------------------------
struct LoadCtx {
    float inv_scale[27];
};
using PoolFn = void (*)(const PoolBox*, const uint32_t*, const PoolMeta*, int);
using GammaFn = void (*)(int, const void*, Geom, Coll, LoadCtx, double*);

// c64: the box is x-blocked in chunks of 64 nodes (a pull sweep may then
// take a kernel with that geometry compiled in)
template <int S, bool GX>
StepFn step_kernel(int variant, int sweep, bool c64);
template <int S>
PoolFn pool_kernel(int variant, int sweep, bool one);   // estimate gamma only
template <int S, bool GX>
GammaFn gamma_kernel(int variant);

}  // namespace kbc
