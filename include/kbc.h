/*
 * kbc.h -- C-ABI of the MI355X D3Q27 KBC lattice Boltzmann library
 * (libkbc.so, built from paper_1507_02518_amd/csrc for gfx950).
 *
 * The library advances the populations of a periodic box with the entropic
 * multi-relaxation (KBC) scheme of Boesch, Chikatamarla & Karlin,
 * "Entropic multi-relaxation lattice Boltzmann scheme for turbulent flows"
 * (arXiv:1507.02518):
 *   - propagation f_i(x + v_i, t+1) = f'_i(x, t) on the periodic lattice
 *     (section I, Eq. Egeneral), D3Q27 velocities and weights (section II);
 *   - per node the collision of section IV: conserved moments, product-form
 *     equilibrium (Eq. entropic_eq), shear part s from table s_parts,
 *     ds = s - s^eq, dh = f - f^eq - ds, stabilizer
 *     gamma = 1/beta - (2 - 1/beta) <ds|dh>/<dh|dh> with the entropic scalar
 *     product <X|Y> = sum_i X_i Y_i / f_i^eq (Eq. result21), and the relaxation
 *     f' = f - beta (2 ds + gamma dh);
 *   - beta from the viscosity, nu = c_s^2 (1/(2 beta) - 1/2), c_s^2 = 1/3
 *     (Eqs. viscosity and sound).
 *
 * Conventions shared by every entry point
 *   - Box shape is {nx, ny, nz}, each >= 1, nx*ny*nz < 2^31.
 *   - Host scalar fields are FP64 [nz][ny][nx] with x fastest; host vector
 *     fields are [3][nz][ny][nx]; host population fields are
 *     [27][nz][ny][nx].  Velocity index i = (vx+1) + 3(vy+1) + 9(vz+1)
 *     (rest population i = 13, opposite direction 26 - i).
 *   - The state at time t is the pre-collision field F(t); one step is the
 *     collision followed by propagation, so F(t+1)_i(x) = F'(t)_i(x - v_i).
 *   - Host pointers are owned by the caller and only read or written during
 *     the call.  Every call that returns host data synchronises the box's
 *     stream; kbc_step only enqueues work.
 *   - Every function returns 0 on success or a negative KBC_E* code; the
 *     message of the last failure on the calling thread is kbc_last_error().
 *     No C++ exception crosses this interface.
 *   - One handle must not be used by two host threads at once.
 */
#ifndef KBC_H
#define KBC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KBC_OK 0
#define KBC_EINVAL (-1)     /* bad argument: shape, nu, dtype, variant, NULL */
#define KBC_ENOMEM (-2)     /* device allocation failed */
#define KBC_EDEVICE (-3)    /* HIP runtime error (message in kbc_last_error) */
#define KBC_EUNSTABLE (-4)  /* |u_a| >= 1 or rho <= 0 at init; non-finite state */
#define KBC_ECAPACITY (-5)  /* pool budget or slots exhausted */
#define KBC_ESTATE (-6)     /* call not valid in the current state */

/* Storage precision of the populations.  KBC_F64 stores f_i in FP64 and
 * collides in FP64.  The deviation forms store f_i - W_i (FP32, or FP16 times
 * a per-direction power-of-two scale fixed at initialisation) and collide in
 * FP32.  KBC_F32_DEV_X stores like KBC_F32_DEV but forms rho, u and
 * f_i - f_i^eq in FP64 before the FP32 collision, which removes the
 * cancellation error of the pure FP32 collision (4 bytes per population
 * either way). */
typedef enum { KBC_F64 = 0, KBC_F32_DEV = 1, KBC_F16_DEV = 2, KBC_F32_DEV_X = 3 } kbc_dtype;

/* Shear part s of the KBC models (section IV): s = d, d+t, d+q or d+t+q
 * built from natural moments (table s_parts), or the same four built from
 * central moments about the node's velocity, s = d~, d~+t~, d~+q~, d~+t~+q~
 * (the population representation in the central basis of the appendix).
 * The paper's simulations use d+t+q.  Every variant moves the same bytes;
 * the central ones do more arithmetic per node. */
typedef enum {
    KBC_S_D = 0, KBC_S_DT = 1, KBC_S_DQ = 2, KBC_S_DTQ = 3,
    KBC_S_CD = 4, KBC_S_CDT = 5, KBC_S_CDQ = 6, KBC_S_CDTQ = 7
} kbc_variant;

/* Streaming pattern: two lattices with pull (gather) propagation, or one
 * lattice updated in place with the AA access pattern.  Results are the
 * same; AA halves the memory footprint. */
typedef enum { KBC_PULL = 0, KBC_AA = 1 } kbc_streaming;

/* Stabilizer gamma (section IV).  KBC_GAMMA_ENTROPIC: the estimate gamma*
 * of Eq. result21 (the paper's scheme).  KBC_GAMMA_FIXED: gamma =
 * gamma_value everywhere (2 = LBGK, 1/beta = regularised LB).
 * KBC_GAMMA_EXACT: the root of the entropy-maximum condition Eq. result1 at
 * every node, found in FP64 from gamma* by solving a fourth-order
 * expansion of the condition about it (one pass of 27 logarithms at almost
 * every node; safeguarded Halley iteration where the expansion is not
 * accurate enough: an ALU-bound kernel);
 * gamma = 2 where <dh|dh> <= gamma_eps rho or where the condition has no
 * root with all post-collision populations positive.  Single boxes only;
 * kbc_pool_create rejects it. */
typedef enum { KBC_GAMMA_ENTROPIC = 0, KBC_GAMMA_FIXED = 1, KBC_GAMMA_EXACT = 2 } kbc_gamma_mode;

typedef struct kbc_options {
    int32_t variant;        /* kbc_variant; default KBC_S_DTQ */
    int32_t streaming;      /* kbc_streaming; default KBC_PULL */
    int32_t gamma_mode;     /* kbc_gamma_mode; default KBC_GAMMA_ENTROPIC */
    int32_t device;         /* HIP device ordinal; -1 = current device */
    double gamma_value;     /* used with KBC_GAMMA_FIXED (2 = LBGK, 1/beta = RLB) */
    double gamma_eps;       /* gamma = 2 where <dh|dh> <= gamma_eps * rho;
                               <= 0 selects the default (1e-28 for FP64,
                               1e-16 for the FP32 collision) */
    void* stream;           /* hipStream_t to enqueue on (borrowed, must outlive
                               the handle); NULL = the library creates one */
} kbc_options;

typedef struct kbc_box* kbc_handle;

/* Fill *opt with the defaults listed above. */
void kbc_options_default(kbc_options* opt);

/* Create a box of shape {nx, ny, nz} with kinematic viscosity nu > 0
 * (beta = 1/(6 nu + 1) in (0, 1)) and the given storage dtype.  opt may be
 * NULL.  Allocates the device population buffers (two lattices for
 * KBC_PULL, one for KBC_AA); the populations are undefined until
 * kbc_init_velocity or kbc_set_populations.  On success *out owns the box.
 * The device layout of the populations is internal (x-blocked for pull boxes
 * whose lattice spans less than 4 GiB, one plane per direction otherwise)
 * and never crosses this interface.  Some calls add device buffers on their
 * first use, kept until kbc_destroy: the velocity field the diagnostics
 * reduce over (24 B per node; 8 B more per node for a density that is read
 * or passed in) for kbc_init_velocity from host memory, kbc_moments,
 * kbc_energy, kbc_energy_series, kbc_enstrophy, kbc_statistics and
 * kbc_correlation; an FP64 copy of the populations (216 B per node) for
 * kbc_get_populations and kbc_set_populations.  kbc_init_velocity_device,
 * kbc_step, kbc_sample_populations, kbc_gamma_statistics and the
 * no-allocation energy series add none of them. */
int kbc_create(const int64_t shape[3], double nu, int32_t dtype,
               const kbc_options* opt, kbc_handle* out);

/* Release every device resource of the box.  NULL is accepted. */
int kbc_destroy(kbc_handle h);

/* F(0) = f^eq(rho, u) at every node (product-form equilibrium, section II),
 * t = 0.  u: host [3][nz][ny][nx] FP64; rho: host [nz][ny][nx] FP64 or NULL
 * for rho = 1.  Returns KBC_EUNSTABLE (state unchanged) if some |u_a| >= 1
 * or rho <= 0, where the equilibrium is not positive. */
int kbc_init_velocity(kbc_handle h, const double* u, const double* rho);

/* Same, with u and rho already in device memory (same layouts). */
int kbc_init_velocity_device(kbc_handle h, const double* u_dev, const double* rho_dev);

/* Enqueue n >= 0 steps on the box's stream and return; t advances by n.
 * Each step is one kernel launch; from n >= 16 on, runs of 16 steps are
 * replayed from a graph the box builds on first use (the same kernels and
 * arguments, so the same results as 16 single launches). */
int kbc_step(kbc_handle h, int64_t n);

/* Density and velocity of F(t) (section I: rho = sum_i f_i, rho u =
 * sum_i v_i f_i) copied to host arrays rho [nz][ny][nx] and u [3][nz][ny][nx];
 * either may be NULL.  Synchronises.  KBC_EUNSTABLE if any value is not
 * finite (the arrays are still written). */
int kbc_moments(kbc_handle h, double* rho, double* u);

/* Kinetic energy k = (1/2) < |u - <u>|^2 > of F(t) (section V), <.> the mean
 * over nodes, reduced in FP64 on the device in a fixed order (bitwise
 * reproducible).  Synchronises.  KBC_EUNSTABLE if the state is not finite. */
int kbc_energy(kbc_handle h, double* k);

/* Advance n >= 0 steps and return the kinetic energy after each of them:
 * k[j] = k of F(t0 + j + 1), j = 0 .. n-1, host FP64 array of n values
 * (NULL allowed when n = 0).  The same reduction as kbc_energy (bitwise equal
 * to calling kbc_step(h, 1) and kbc_energy after every step), but enqueued
 * with the steps and copied back once at the end; allocates and frees a
 * device array of n doubles.  Synchronises.  KBC_EUNSTABLE if the state was
 * not finite after some step (the steps are taken and k is still written). */
int kbc_energy_series(kbc_handle h, int64_t n, double* k);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc, such as a tight serving loop or a harness that forbids it):
 * kbc_energy_series without any allocation.  Advances n steps and writes the
 * kinetic energy after each of them to host k[0 .. n-1], as kbc_energy_series
 * does (the same sums in the same order), but reads the velocity straight
 * from the populations and keeps its partial sums and the log of k in a
 * static device array of the library instead of device buffers:
 * 0 <= n <= KBC_NOALLOC_MAX_STEPS, else KBC_EINVAL.  The array (about 540 KB)
 * exists once per GPU the library runs on and is held until the process
 * ends; its address is looked up on the first call on each device.  Every
 * call on a GPU uses that GPU's array, so calls that overlap on one GPU (from
 * two host threads, or on two boxes whose streams run concurrently) race and
 * must be serialised by the caller.  Synchronises the box's stream.
 * KBC_EUNSTABLE if some k is not finite (the state diverged; k is still
 * written). */
#define KBC_NOALLOC_MAX_STEPS 65536
int kbc_energy_series_noalloc(kbc_handle h, int64_t n, double* k);

/* Enstrophy Omega = (1/2) < |curl u'|^2 >, u' = u - <u>, derivatives by
 * second-order central differences on the periodic grid (section V.A).
 * FP64, fixed reduction order.  Synchronises. */
int kbc_enstrophy(kbc_handle h, double* omega);

/* One-point statistics of section V.A for the velocity of F(t), all means
 * over nodes, derivatives by central differences (order 2 or the nine-point
 * eighth-order stencil the paper uses for its table of statistics), FP64,
 * fixed reduction order:
 *   k          = (1/2) <|u'|^2>
 *   omega      = (1/2) <|curl u'|^2>
 *   epsilon    = (nu/2) <(d_a u'_b + d_b u'_a)(d_a u'_b + d_b u'_a)>
 *   div2       = <(div u)^2>  (epsilon - 2 nu omega = 2 nu div2 exactly)
 *   dudx_moment[n-2] = <(d u'_x / dx)^n>, n = 2..6
 *   skewness[n-3]    = (-1)^n <(du'_x/dx)^n> / <(du'_x/dx)^2>^(n/2), n = 3..6
 * The derived turbulence, Taylor and Kolmogorov scales follow from k,
 * epsilon and nu on the host. */
typedef struct kbc_stats {
    double k, omega, epsilon, div2;
    double dudx_moment[5];
    double skewness[4];
} kbc_stats;

/* Fill *out for the current state.  order: 2 or 8 (KBC_EINVAL otherwise).
 * KBC_EUNSTABLE if the state is not finite.  Synchronises. */
int kbc_statistics(kbc_handle h, int32_t order, kbc_stats* out);

/* Statistics of the stabilizer gamma (section V.C) that the next step
 * applies at each node (the collision evaluated on F(t), nothing written):
 * out[0] mean, out[1] standard deviation, out[2] minimum, out[3] maximum
 * over the nodes.  Follows the box's variant and gamma mode (a fixed gamma
 * gives mean = gamma, std = 0).  Synchronises. */
int kbc_gamma_statistics(kbc_handle h, double out[4]);

/* Longitudinal and transversal velocity correlations along x (section
 * V.B): rho11[r] = <u'_x(x) u'_x(x + r)> / <u'_x^2>,
 * rho22[r] = <u'_y(x) u'_y(x + r)> / <u'_y^2>, r = 0..rmax (host arrays of
 * rmax + 1).  Requires nx <= 4096 and 0 <= rmax < nx.  Allocates and frees
 * a small device buffer.  Synchronises. */
int kbc_correlation(kbc_handle h, int32_t rmax, double* rho11, double* rho22);

/* Copy F(t) to host f [27][nz][ny][nx] FP64 (deviation storage is decoded
 * to full populations).  Synchronises. */
int kbc_get_populations(kbc_handle h, double* f);

/* Copy F(t) at `count` selected nodes to host f [count][27] FP64.  nodes
 * holds linear node indices (x + nx*(y + ny*z)), each in [0, nx*ny*nz);
 * returns KBC_EINVAL (nothing copied) if one is out of range.  Synchronises.
 * Lets a caller check a large box at a few nodes without copying it whole. */
int kbc_sample_populations(kbc_handle h, const int64_t* nodes, int64_t count, double* f);

/* Replace the state by host f [27][nz][ny][nx] FP64 taken as F(t), and set
 * the step counter to t >= 0.  Deviation storage rounds f_i - W_i to the
 * storage precision (FP16 keeps the scales chosen at initialisation, or
 * picks them from f when the box was never initialised). */
int kbc_set_populations(kbc_handle h, const double* f, int64_t t);

/* Current step counter. */
int kbc_time(kbc_handle h, int64_t* t);

/* Wait for every step enqueued on the box's stream. */
int kbc_sync(kbc_handle h);

/* HBM bytes one step moves per lattice node if each population is read and
 * written exactly once (2 * 27 * bytes per stored population). */
int kbc_bytes_per_node_step(kbc_handle h, double* bytes);

/* The stream the box enqueues on (a hipStream_t). */
int kbc_stream(kbc_handle h, void** stream);

/* ------------------------------------------------------------------------
 * Batched ensemble ("pool"): continuous batching of many independent boxes.
 *
 * A pool owns an HBM arena of hbm_budget_bytes.  Each admitted box (any
 * shape, its own viscosity and step count) takes 27 * N * bytes-per-
 * population of it and is updated in place with the AA pattern.  One
 * kbc_pool_advance(g) enqueues up to g steps for every unfinished box at once
 * (replayed from a captured hipGraph), so boxes admitted while others run
 * share the GPU from their first step on.  The boxes of a batch are split
 * into launch groups of one AA parity whose populations fit the GPU's
 * last-level cache; a group takes all its steps of the batch, one launch per
 * step, before the next group starts.  Each box evolves exactly as the same box alone (same
 * kernels, same arithmetic), so results do not depend on the mix.  Launch
 * shape (threads per block, blocks: one per tile or a persistent grid,
 * block-sized sub-tiles per tile) comes from an online autotuner.  Batches
 * are classed by floor(log2(mean nodes per box)); the first batches of a new
 * class time each of 12 candidate shapes twice on real work, and the fastest
 * is kept for that class (and per dtype and variant in the text file
 * tune_cache, which may be NULL).  Batches of a class still being measured
 * by another round run one block per tile, 256 threads.
 * ------------------------------------------------------------------------ */
typedef struct kbc_pool* kbc_pool_handle;

/* Create a pool.  dtype and opt (variant, gamma options, device, stream) as
 * for kbc_create; opt->streaming is ignored.  max_slots in [1, 65536] bounds
 * the number of resident boxes.  KBC_ENOMEM if the arena cannot be had. */
int kbc_pool_create(size_t hbm_budget_bytes, int32_t dtype, const kbc_options* opt,
                    int32_t max_slots, const char* tune_cache, kbc_pool_handle* out);

/* Wait for all work and release every resource.  NULL is accepted. */
int kbc_pool_destroy(kbc_pool_handle p);

/* Admit a box of shape {nx, ny, nz}, viscosity nu, initial velocity u (host
 * [3][nz][ny][nx] FP64, rho = 1) that will run `steps` steps.  Returns its
 * slot in *slot.  KBC_ECAPACITY (nothing changed) if no slot is free or the
 * arena has no contiguous room; KBC_EUNSTABLE if some |u_a| >= 1.
 * Synchronises only with the pool's own admission stream, not with running
 * batches. */
int kbc_pool_admit(kbc_pool_handle p, const int64_t shape[3], double nu, const double* u,
                   int64_t steps, int32_t* slot);

/* Enqueue a batch: every resident box with steps left runs min(g, left)
 * steps, g in [1, 4096].  Returns without waiting. */
int kbc_pool_advance(kbc_pool_handle p, int64_t g);

/* Same, for the listed slots only (count >= 0; the others wait): lets a
 * scheduler order the work, e.g. shortest remaining work first.  KBC_EINVAL
 * if a listed slot is empty. */
int kbc_pool_advance_slots(kbc_pool_handle p, int64_t g, const int32_t* slots, int32_t count);

/* Steps of the box not yet completed on the device (0 = result ready).
 * Does not block. */
int kbc_pool_poll(kbc_pool_handle p, int32_t slot, int64_t* remaining);

/* For a box that has run all its steps: kinetic energy k and enstrophy Omega
 * (as kbc_energy / kbc_enstrophy) and optionally rho [nz][ny][nx] and
 * u [3][nz][ny][nx] (host, may be NULL).  Waits for the box's last batch
 * only.  KBC_ESTATE if steps are left; KBC_EUNSTABLE if the state is not
 * finite (other boxes are unaffected). */
int kbc_pool_result(kbc_pool_handle p, int32_t slot, double* k, double* omega, double* rho,
                    double* u);

/* Free the box's slot and arena region (waits for its last batch). */
int kbc_pool_release(kbc_pool_handle p, int32_t slot);

/* Wait for every enqueued batch. */
int kbc_pool_sync(kbc_pool_handle p);

/* Arena bytes in use, resident boxes, the launch shape of the latest batch
 * (threads per block; blocks, 0 meaning one block per tile; block-sized
 * sub-tiles per tile) and whether a tuning round is in progress (any pointer
 * may be NULL). */
int kbc_pool_info(kbc_pool_handle p, size_t* bytes_used, int32_t* boxes, int32_t* block,
                  int32_t* grid, int32_t* sub, int32_t* tuning);

/* Fix the launch shape for every batch (block: 64..512 in steps of 64;
 * grid >= 0, 0 for one block per tile; sub in 1..64) and stop tuning. */
int kbc_pool_set_launch(kbc_pool_handle p, int32_t block, int32_t grid, int32_t sub);

/* Measurement utility (not part of the method): copy `bytes` (a multiple of
 * 16) from device src to device dst with a plain streaming kernel on the
 * given hipStream_t (NULL = default stream), without synchronising.  Its
 * duration and HBM counters give the achievable copy bandwidth and the
 * scale of the rocprof FETCH_SIZE / WRITE_SIZE counters against known bytes.
 * With dst == src every 16-byte word is read and written back unchanged at
 * its own address (the traffic of an in-place sweep, which streams slower
 * than a copy between two buffers); other overlapping ranges are rejected
 * (KBC_EINVAL). */
int kbc_hbm_copy(void* dst, const void* src, size_t bytes, void* stream);

/* Message of the last failed call on this thread ("" if none).  Valid until
 * the next failing call on the same thread. */
const char* kbc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* KBC_H */
