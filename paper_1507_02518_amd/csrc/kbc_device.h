// kbc_device.h -- device-side definitions of the D3Q27 KBC update for gfx950:
// lattice constants, index helpers, kernel parameter blocks, storage codecs
// and the per-node collision of section IV of Boesch, Chikatamarla & Karlin
// (arXiv:1507.02518).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kbc {

enum Storage : int { ST_F64 = 0, ST_F32 = 1, ST_F16 = 2, ST_F32X = 3 };
// s = d, d+t, d+q, d+t+q from natural moments (table s_parts), and the same
// four from central moments (section IV; appendix)
enum Variant : int {
    V_D = 0, V_DT = 1, V_DQ = 2, V_DTQ = 3,
    V_CD = 4, V_CDT = 5, V_CDQ = 6, V_CDTQ = 7
};
__host__ __device__ constexpr bool is_central(int v) { return v >= V_CD; }
__host__ __device__ constexpr bool with_t(int v)
{
    return v == V_DT || v == V_DTQ || v == V_CDT || v == V_CDTQ;
}
__host__ __device__ constexpr bool with_q(int v)
{
    return v == V_DQ || v == V_DTQ || v == V_CDQ || v == V_CDTQ;
}
enum Sweep : int { SW_PULL = 0, SW_AA_EVEN = 1, SW_AA_ODD = 2 };

// D3Q27 velocities: tensor product of three copies of {-1, 0, 1}
// (section II).  Direction i = (vx+1) + 3(vy+1) + 9(vz+1); opposite 26-i.
__host__ __device__ constexpr int vel(int i, int a)
{
    return a == 0 ? i % 3 - 1 : (a == 1 ? (i / 3) % 3 - 1 : i / 9 - 1);
}
__host__ __device__ constexpr int opp(int i) { return 26 - i; }

// One-dimensional weights W_0 = 2/3, W_{+-1} = 1/6; D3Q27 weight is their
// product over the three axes (section II).
__host__ __device__ constexpr double w1(int c) { return c == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }
__host__ __device__ constexpr double weight(int i)
{
    return w1(vel(i, 0)) * w1(vel(i, 1)) * w1(vel(i, 2));
}

// Division of a node index n < 2^31 by a runtime divisor d >= 1 with one
// high multiply, an add and a shift (round-up magic number, shift ceil(log2 d)).
struct FastDiv {
    uint32_t d, m, s;
};

inline FastDiv make_fastdiv(uint32_t d)
{
    uint32_t s = 0;
    while ((uint64_t(1) << s) < d) ++s;
    const uint64_t m = ((uint64_t(1) << 32) * ((uint64_t(1) << s) - d)) / d + 1;
    return FastDiv{d, (uint32_t)m, s};
}

__host__ __device__ inline uint32_t fdiv(uint32_t n, const FastDiv& f)
{
#if defined(__HIP_DEVICE_COMPILE__)
    const uint32_t hi = __umulhi(n, f.m);
#else
    const uint32_t hi = (uint32_t)(((uint64_t)n * f.m) >> 32);
#endif
    return (hi + n) >> f.s;
}

// Geometry of one periodic box inside a population buffer, and where
// population slot s of node (x, y, z) sits in it: element
//   s * plane + z * slab + y * row + (x >> xshift) * chunk + (x & xmask).
// Two layouts use this form:
//   planes    [27][nz][ny][nx] (plane >= nnodes, row = nx, slab = nx*ny,
//             xshift = 31, so a row is one chunk and x & xmask = x);
//   x-blocked [nz][ny][nx/B][27][B] (plane = B, chunk = 27 B, row = 27 nx,
//             slab = 27 nx ny, B = 2^xshift, xmask = B - 1; with B = nx and
//             xshift = 31 for rows that no power of two >= 32 divides).
struct Geom {
    uint32_t nx, ny, nz, nnodes;   // nnodes = nx*ny*nz
    FastDiv dnx, dny;
    uint64_t plane;                // elements between consecutive slots
    uint32_t row, slab;            // elements between y and z neighbours
    uint32_t chunk;                // elements between consecutive x-chunks
    uint32_t xshift, xmask;        // chunk and position of x in it
};

__host__ __device__ __forceinline__ uint64_t pop_index(const Geom& g, int slot, uint32_t x,
                                                       uint32_t y, uint32_t z)
{
    return (uint64_t)slot * g.plane + (uint64_t)z * g.slab + (uint64_t)y * g.row +
           (uint64_t)(x >> g.xshift) * g.chunk + (x & g.xmask);
}

// Per-box collision constants.
struct Coll {
    double beta;       // relaxation parameter, nu = (1/3)(1/(2 beta) - 1/2)
    double inv_beta;   // 1/beta
    double c2;         // 2 - 1/beta
    double gamma_eps;  // gamma = 2 where <dh|dh> <= gamma_eps * rho
    double gamma_value;
    int32_t gamma_fixed;
    int32_t pad_;
};

// Orders of a launch's workgroups over the eight XCDs (see step_block).
enum XcdOrder : uint32_t { ORDER_PLAIN = 0, ORDER_PAIRS = 1, ORDER_EIGHTHS = 2 };

struct StepParams {
    const void* src;
    void* dst;
    Geom g;
    Coll c;
    // FP16 storage: stored = (f - W) * 2^scale_exp[i]; zero for the other forms
    int8_t scale_exp[28];
    // order of the workgroups over the XCDs in the AA sweeps (step_block):
    // ORDER_PAIRS or ORDER_EIGHTHS, set by the host per box
    uint32_t xcd_order;
};

__host__ __device__ __forceinline__ float ldexp_(float x, int e)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_ldexpf(x, e);
#else
    return __builtin_ldexpf(x, e);
#endif
}

__device__ inline void node_xyz(uint32_t n, const Geom& g, uint32_t& x, uint32_t& y, uint32_t& z)
{
    const uint32_t yz = fdiv(n, g.dnx);
    x = n - yz * g.nx;
    z = fdiv(yz, g.dny);
    y = yz - z * g.ny;
}

// ---------------------------------------------------------------------------
// Storage codecs.  F64 stores f_i; F32 stores f_i - W_i; F16 stores
// (f_i - W_i) * scale_i rounded to nearest even.  The arithmetic type R is
// the collision precision; deviation forms collide on g_i = f_i - W_i.
// ---------------------------------------------------------------------------
template <int S> struct Traits;
template <> struct Traits<ST_F64> {
    using T = double;
    using R = double;
    static constexpr bool kDev = false;
    static constexpr bool kMixed = false;
};
template <> struct Traits<ST_F32> {
    using T = float;
    using R = float;
    static constexpr bool kDev = true;
    static constexpr bool kMixed = false;
};
template <> struct Traits<ST_F16> {
    using T = _Float16;
    using R = float;
    static constexpr bool kDev = true;
    static constexpr bool kMixed = false;
};
// FP32 deviation storage; the conserved moments and f - f^eq are formed in
// FP64 (they are differences of O(u) quantities), the rest in FP32.
template <> struct Traits<ST_F32X> {
    using T = float;
    using R = float;
    static constexpr bool kDev = true;
    static constexpr bool kMixed = true;
};

template <int S>
__device__ __forceinline__ typename Traits<S>::R decode(typename Traits<S>::T v, float inv_scale)
{
    if constexpr (S == ST_F16) return (float)v * inv_scale;
    else return v;
}

// The step kernels scale FP16 deviations by powers of two held as exponents
// (a byte per direction rather than two floats): ldexp equals the
// multiplication by 2^e exactly, so both codecs give the same bits.
template <int S>
__device__ __forceinline__ typename Traits<S>::R decode_exp(typename Traits<S>::T v, int e)
{
    if constexpr (S == ST_F16) return ldexp_((float)v, -e);
    else return v;
}

template <int S>
__device__ __forceinline__ typename Traits<S>::T encode_exp(typename Traits<S>::R v, int e)
{
    if constexpr (S == ST_F16) return (_Float16)ldexp_(v, e);
    else return v;
}

template <int S>
__device__ __forceinline__ typename Traits<S>::T encode(typename Traits<S>::R v, float scale)
{
    if constexpr (S == ST_F16) return (_Float16)(v * scale);
    else return v;
}

// ---------------------------------------------------------------------------
// Collision of one node, in place on f[27] (f_i for F64, g_i = f_i - W_i for
// the deviation forms): the KBC mirror state of section IV inserted in
// Eq. Egeneral, f' = f - beta (2 ds + gamma dh).
//   - rho and u from a separable 3x3x3 moment transform of f;
//   - f^eq (Eq. entropic_eq) from its one-dimensional marginals: with
//     S = sqrt(1+3u^2) the product-form factors reduce to e_0 = (4 - 2S)/3,
//     e_{+-1} = ((2S - 1)/3 +- u)/2 per axis, f_i^eq = rho e(vx) e(vy) e(vz);
//   - ds = s - s^eq from the differences of the 13 second- and third-order
//     natural moments of f and f^eq (table s_parts), or, for the central
//     variants, from the central moments of those differences (appendix);
//   - dh = f - f^eq - ds (Eq. ksh-representation: the kinematic part
//     depends only on rho and u, so it cancels);
//   - gamma = 1/beta - (2 - 1/beta) <ds|dh>/<dh|dh> (Eq. result21),
//     1/f^eq_i separable; gamma = 2 where <dh|dh> <= gamma_eps * rho (0/0
//     at equilibrium).
// ---------------------------------------------------------------------------

// Separable moment transform along x, then y, then z: for each line of three
// populations (v = -1, 0, +1) the sums m0 = f- + f0 + f+, m1 = f+ - f-,
// m2 = f+ + f-.  M[p][q][r] = sum_i g_i vx^p vy^q vz^r.
template <typename R>
__host__ __device__ __forceinline__ void moments27(const R (&g)[27], R (&M)[3][3][3])
{
    R X[3][9];
#pragma unroll
    for (int yz = 0; yz < 9; ++yz) {
        const R fm = g[3 * yz + 0], f0 = g[3 * yz + 1], fp = g[3 * yz + 2];
        const R s2 = fp + fm;
        X[0][yz] = s2 + f0;
        X[1][yz] = fp - fm;
        X[2][yz] = s2;
    }
    R Y[3][3][3];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int az = 0; az < 3; ++az) {
            const R a = X[p][3 * az + 0], b = X[p][3 * az + 1], d = X[p][3 * az + 2];
            const R s2 = d + a;
            Y[p][0][az] = s2 + b;
            Y[p][1][az] = d - a;
            Y[p][2][az] = s2;
        }
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const R a = Y[p][q][0], b = Y[p][q][1], d = Y[p][q][2];
            const R s2 = d + a;
            M[p][q][0] = s2 + b;
            M[p][q][1] = d - a;
            M[p][q][2] = s2;
        }
}

// Differences of the named moments of section III between f and f^eq, plus
// the three diagonal second moments (T, N_xz, N_yz are combinations of them).
template <typename R>
struct DMom {
    R T, Nxz, Nyz, Pxy, Pxz, Pyz, Qxyy, Qxzz, Qxxy, Qyzz, Qxxz, Qyyz, Qxyz;
    R Dxx, Dyy, Dzz;
};

// Reciprocal and square root: IEEE-exact in FP64; in the FP32 collision the
// hardware approximations (about 1 ulp), far below that path's own error.
__host__ __device__ __forceinline__ double rcp_(double x) { return 1.0 / x; }
__host__ __device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
__host__ __device__ __forceinline__ float rcp_(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}
__host__ __device__ __forceinline__ float sqrt_(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_sqrtf(x);
#else
    return sqrtf(x);
#endif
}

// One-dimensional equilibrium marginals of one axis (section II, product
// form): e[v+1] and de[v+1] = e - W_v, plus m2 - 1/3 where m2 = (2S - 1)/3.
template <typename R, bool kNoCancel>
__host__ __device__ __forceinline__ void marginals1d(R u, R (&e)[3], R (&de)[3], R& dm2)
{
    const R q3 = R(3) * u * u;
    const R Sq = sqrt_(R(1) + q3);
    R sm1;  // S - 1, without cancellation where asked
    if constexpr (kNoCancel) sm1 = q3 * rcp_(R(1) + Sq);
    else sm1 = Sq - R(1);
    dm2 = R(2.0 / 3.0) * sm1;
    const R half_u = R(0.5) * u;
    de[1] = -dm2;
    de[2] = R(0.5) * dm2 + half_u;
    de[0] = R(0.5) * dm2 - half_u;
    e[1] = R(2.0 / 3.0) + de[1];
    e[2] = R(1.0 / 6.0) + de[2];
    e[0] = R(1.0 / 6.0) + de[0];
}

// 1/e for the three marginal values of one axis from a single division.
template <typename R>
__host__ __device__ __forceinline__ void recip3(const R (&e)[3], R (&ie)[3])
{
    const R pm = e[0] * e[2];
    const R ip = rcp_(pm * e[1]);
    ie[1] = pm * ip;
    ie[2] = e[1] * e[0] * ip;
    ie[0] = e[1] * e[2] * ip;
}

// ln(1 + x) near zero, where the arguments of the exact stabilizer lie in all
// but strongly non-equilibrium states: x P(x), with P the degree-9
// Chebyshev economization (Lanczos) of the Taylor series of ln(1 + x) / x =
// 1 - x/2 + x^2/3 - ... on |x| <= 1/16: the series in t = 16 x, rewritten in
// Chebyshev polynomials T_k(t), cut after T_9 and converted back to powers
// of x.  The dropped Chebyshev coefficients sum to 1.7e-16, so the relative
// error of x P(x) evaluated in FP64 stays below 4e-16 there (about two ulp,
// as the library function): four fused multiply-adds fewer than the plain
// Taylor series of the same accuracy.  log1p_ takes the library log1p
// elsewhere.
__host__ __device__ __forceinline__ double log1p_series(double x)
{
    constexpr double c[10] = {0x1.0000000000001p+0,  -0x1.0000000000007p-1,
                              0x1.555555554c29ap-2,  -0x1.ffffffffdafbap-3,
                              0x1.99999a2c404b2p-3,  -0x1.55555624817afp-3,
                              0x1.2490aee4998aep-3,  -0x1.fffc4ddce731dp-4,
                              0x1.cac4744a4f262p-4,  -0x1.9d49ddb1b5841p-4};
    double p = c[9];
#pragma unroll
    for (int k = 8; k >= 0; --k) p = fma(p, x, c[k]);
    return x * p;
}

__host__ __device__ __forceinline__ bool log1p_series_ok(double x) { return fabs(x) < 0.0625; }

__host__ __device__ __forceinline__ double log1p_(double x)
{
    return log1p_series_ok(x) ? log1p_series(x) : log1p(x);
}

// 1/x from the hardware estimate refined by Newton steps (x is a positive
// normal number here), in place of an IEEE division: two steps take the
// estimate (relative error near 2^-23) to about one ulp, one step to about
// 2^-46.
template <int STEPS = 2>
__host__ __device__ __forceinline__ double rcp_refined_(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rcp(x);
#pragma unroll
    for (int k = 0; k < STEPS; ++k) r = fma(r, fma(-x, r, 1.0), r);
    return r;
#else
    return 1.0 / x;
#endif
}

// Exact stabilizer (section IV, Eq. result1): the root in gamma of
//   G(gamma) = sum_i dh_i ln(1 + x_i),  x_i = ((1 - beta gamma) dh_i - (2 beta - 1) ds_i) / f^eq_i,
// where 1 + x_i = f'_i / f^eq_i.  The caller passes, per population, dh_i,
// hw_i = dh_i / f^eq_i and cc_i = (dh_i - (2 beta - 1) ds_i) / f^eq_i, so that
// x_i = cc_i - beta gamma hw_i.  With r_i = hw_i / (1 + x_i) and
// M_k = sum_i dh_i r_i^k,
//   G'  = -beta   M_1,   G'' = -beta^2 M_2,
// and, exactly, G(gamma + d) = G(gamma) - sum_{k>=1} (beta d)^k M_k / k.
// On the interval where all 1 + x_i are positive G falls strictly (M_1 > 0),
// so the root there is unique.  Each pass over the populations (from the
// estimate g0 first) forms G and M_1..M_4 and solves the expansion cut after
// k = 4 for d by Newton's method from Halley's step; with q = |beta d| max r_i
// the dropped terms move that root by at most |d| q^4 / (5 (1 - q)), and when
// that is below the tolerance the pass ends the search.  Otherwise Halley's
// step 2 G M_1 / (beta (2 M_1^2 + G M_2)) (Newton's G / (beta M_1) where
// |G M_2| > M_1^2) is taken and the pass repeated, each iterate kept inside
// a bracket that shrinks with the sign of G (a step that leaves it is
// replaced by bisection); FP64 for every storage form.  A change dg of gamma
// moves f'_i by beta dg dh_i, so the search stops once the last correction
// moves no population by more than 1e-16 f^eq_i: further digits of gamma
// cannot change the result, and where dh << ds they are not determined by G
// to begin with.  Two Halley steps in a row bound the next one (at least
// quadratic convergence: s_{n+1} <~ s_n^3 / s_{n-1}^2), and when that bound
// is already below the tolerance the search stops without evaluating G
// again.  From gamma* (first-order accurate) one pass suffices at almost
// every node.  Returns false, leaving gamma to the caller, when no bracket
// exists.
__host__ __device__ inline bool gamma_exact_root(const double (&dh)[27], const double (&hw)[27],
                                                 const double (&cc)[27], double beta, double g0,
                                                 double& gamma)
{
    const double inf = __builtin_inf();
    double lo = -inf, hi = inf, hmax = 0.0;
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        // 1 + x_i > 0  <=>  beta gamma hw_i < 1 + cc_i (hw_i has the sign of
        // dh_i; where it is 0 the population gives no bound); no branches, so
        // that the 27 terms stay one block of code
        // The bound comes from a reciprocal refined once (relative error
        // near 2^-44) moved inward by 2^-40 of itself, so it never lies
        // outside the exact one; the root is far inside (G runs to -inf /
        // +inf at the ends).
        hmax = fmax(hmax, fabs(hw[i]));
        const double ah = fabs(beta * hw[i]);
        const double b = (1.0 + cc[i]) * rcp_refined_<1>(ah);   // bound on +-gamma
        const double shrink = fabs(b) * 0x1p-40;
        hi = hw[i] > 0.0 ? fmin(hi, b - shrink) : hi;
        lo = hw[i] < 0.0 ? fmax(lo, -b + shrink) : lo;
    }
    if (!(lo < hi) || !(lo > -inf) || !(hi < inf)) return false;
    double g = (g0 > lo && g0 < hi) ? g0 : 0.5 * (lo + hi);
    const double dg_tol = 1e-16 / (beta * hmax);
    double prev = 0.0;   // size of the last step (0: none yet)
    for (int it = 0; it < 80; ++it) {
        // G by the series wherever it holds (no branch per population: one
        // block of straight code); a node with some |x_i| >= 1/16 sums G
        // again with the library logarithm.  With r_i = hw_i / (1 + x_i) the
        // same pass forms M_k = sum_i dh_i r_i^k, k = 1..4 (each term of M_1
        // is dh_i^2 / (f^eq_i (1 + x_i)) >= 0, so |M_k| <= rmax^(k-1) M_1).
        double G = 0.0, M1 = 0.0, M2 = 0.0, M3 = 0.0, M4 = 0.0, rmax = 0.0;
        bool series = true;
        const double bg = beta * g;
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            const double x = cc[i] - bg * hw[i];
            series = series && log1p_series_ok(x);
            G += dh[i] * log1p_series(x);
            const double r = hw[i] * rcp_refined_(1.0 + x);
            const double t1 = dh[i] * r, t2 = t1 * r, t3 = t2 * r;
            M1 += t1;
            M2 += t2;
            M3 += t3;
            M4 += t3 * r;
            rmax = fmax(rmax, fabs(r));
        }
        if (!series) {
            G = 0.0;
#pragma unroll
            for (int i = 0; i < 27; ++i) G += dh[i] * log1p_(cc[i] - bg * hw[i]);
        }
        if (G == 0.0) break;
        if (G > 0.0) lo = g;
        else hi = g;
        // Halley's step from G, G' = -beta M1, G'' = -beta^2 M2
        const double GD2 = G * M2, D1s = M1 * M1;
        const double step = fabs(GD2) <= D1s ? 2.0 * G * M1 / (beta * (2.0 * D1s + GD2))
                                             : G / (beta * M1);
        // About g, ln(1 + x_i - beta d hw_i) = ln(1 + x_i) + ln(1 - beta d r_i),
        // so G(g + d) = G - sum_k (beta d)^k M_k / k.  The root d of the
        // expansion to k = 4 (Newton from Halley's step) is the root of G to
        // within |d| q^4 / (5 (1 - q)), q = |beta d| rmax; where that is below
        // the tolerance one pass over the populations has found gamma.
        double d = step;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double y = beta * d;
            const double P = G - y * (M1 + y * (0.5 * M2 + y * ((1.0 / 3.0) * M3 + 0.25 * y * M4)));
            const double dP = -beta * (M1 + y * (M2 + y * (M3 + y * M4)));
            d -= P / dP;
        }
        const double q = fabs(beta * d) * rmax, q2 = q * q;
        if (q < 0.25 && fabs(d) * q2 * q2 <= 4.0 * dg_tol * (1.0 - q)) {
            const double gn = g + d;
            if (gn > lo && gn < hi) {
                g = gn;
                break;
            }
        }
        const double as = fabs(step);
        if (as <= dg_tol ||                      // converged (also when the step
            (prev > 0.0 && as < prev &&          // is below one ulp of g), or
             as * as * as <= dg_tol * prev * prev)) {   // the next one would be
            g += step;
            break;
        }
        double gn = g + step;
        if (!(gn > lo && gn < hi)) {
            gn = 0.5 * (lo + hi);
            prev = 0.0;
        } else {
            prev = as;
        }
        g = gn;
    }
    gamma = g;
    return true;
}

// dh, gamma and the relaxation, given ds_i (ds_of(i)), f - f^eq (fneq_of(i))
// and the separable 1/f^eq = iCx[vx+1] * iA9[(vy+1) + 3(vz+1)].  GX selects
// the exact stabilizer (root of Eq. result1) in place of the estimate gamma*;
// it then also needs the equilibrium in the stored form (eq_of(i): f^eq_i,
// or f^eq_i - W_i for the deviation forms, DEV) and in FP64 product form.
template <typename R, bool GX, bool DEV = false, typename DsFn, typename FneqFn,
          typename EqFn = int>
__host__ __device__ __forceinline__ void kbc_gamma_relax(R (&f)[27], DsFn ds_of, FneqFn fneq_of,
                                                         const R (&iCx)[3], const R (&iA9)[9],
                                                         double rho, const Coll& c, double* gout,
                                                         EqFn eq_of = 0)
{
    if constexpr (GX) {
        // The exact root iterates on three FP64 values per population, formed
        // once here; f itself is not needed again: with x_i = cc_i -
        // beta gamma hw_i the post-collision population is
        // f'_i = f^eq_i (1 + x_i) = f_i - beta (2 ds_i + gamma dh_i), so it is
        // rebuilt from the equilibrium, which keeps the live state small.
        double dh[27], hw[27], cc[27];
        R sh = R(0), hh = R(0);
        const double a = 2.0 * c.beta - 1.0;
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            const R ds = ds_of(i);
            const R fneq = fneq_of(i);
            const R w = iCx[i % 3] * iA9[i / 3];
            const R wr = (fneq - ds) * w;
            sh += ds * wr;
            hh += (fneq - ds) * wr;
            const double dsd = (double)ds, wd = (double)w;
            dh[i] = (double)fneq - dsd;
            hw[i] = dh[i] * wd;
            cc[i] = (dh[i] - a * dsd) * wd;
        }
        double gamma;
        if (c.gamma_fixed) {
            gamma = c.gamma_value;
        } else if ((double)hh <= c.gamma_eps * rho) {
            gamma = 2.0;
        } else {
            const double g0 = c.inv_beta - c.c2 * (double)sh / (double)hh;
            double ge;
            gamma = gamma_exact_root(dh, hw, cc, c.beta, g0, ge) ? ge : 2.0;
        }
        if (gout) *gout = gamma;
        const double bg = c.beta * gamma;
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            const double eq = eq_of(i);
            const double feq = DEV ? eq + weight(i) : eq;
            f[i] = R(eq + feq * (cc[i] - bg * hw[i]));
        }
        return;
    } else {
        // dh and the entropic scalar products of Eq. result21
        R sh = R(0), hh = R(0);
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            const R ds = ds_of(i);
            const R dh = fneq_of(i) - ds;
            const R w = dh * (iCx[i % 3] * iA9[i / 3]);
            sh += ds * w;
            hh += dh * w;
        }
        R gamma;
        if (c.gamma_fixed) {
            gamma = R(c.gamma_value);
        } else {
            // ratio and fallback test in FP64 for every storage form
            const double hhd = (double)hh, shd = (double)sh;
            if (hhd <= c.gamma_eps * rho) gamma = R(2);
            else gamma = R(c.inv_beta - c.c2 * shd / hhd);
        }

        if (gout) *gout = (double)gamma;

        // relaxation f' = f - beta (2 ds + gamma dh) (Eq. Egeneral with the
        // mirror state of Eq. ksh-mirror), evaluated with dh = (f - f^eq) - ds
        // as f' = f - beta (2 - gamma) ds - beta gamma (f - f^eq)
        const R c1 = R(c.beta) * (R(2) - gamma);
        const R c2 = R(c.beta) * gamma;
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            const R ds = ds_of(i);
            const R fneq = fneq_of(i);
            f[i] = f[i] - c1 * ds - c2 * fneq;
        }
    }
}

// Natural-moment variants: ds_i from table s_parts, then kbc_gamma_relax.
template <typename R, int V, bool GX, bool DEV, typename FneqFn, typename EqFn>
__host__ __device__ __forceinline__ void kbc_relax(R (&f)[27], const DMom<R>& d, FneqFn fneq_of,
                                                   const R (&iCx)[3], const R (&iA9)[9],
                                                   double rho, const Coll& c, double* gout,
                                                   EqFn eq_of)
{
    constexpr bool WT = with_t(V);
    constexpr bool WQ = with_q(V);
    // table s_parts: value of ds per direction class
    const R t6 = WT ? d.T * R(1.0 / 6.0) : R(0);
    const R sRest = WT ? -d.T : R(0);
    const R sF[3] = {(R(2) * d.Nxz - d.Nyz) * R(1.0 / 6.0) + t6,
                     (R(2) * d.Nyz - d.Nxz) * R(1.0 / 6.0) + t6,
                     -(d.Nxz + d.Nyz) * R(1.0 / 6.0) + t6};
    const R qF[3] = {WQ ? R(-0.5) * (d.Qxyy + d.Qxzz) : R(0),
                     WQ ? R(-0.5) * (d.Qxxy + d.Qyzz) : R(0),
                     WQ ? R(-0.5) * (d.Qxxz + d.Qyyz) : R(0)};
    const R eXY = R(0.25) * d.Pxy, eXZ = R(0.25) * d.Pxz, eYZ = R(0.25) * d.Pyz;
    const R qXYy = WQ ? R(0.25) * d.Qxxy : R(0), qXYx = WQ ? R(0.25) * d.Qxyy : R(0);
    const R qXZz = WQ ? R(0.25) * d.Qxxz : R(0), qXZx = WQ ? R(0.25) * d.Qxzz : R(0);
    const R qYZz = WQ ? R(0.25) * d.Qyyz : R(0), qYZy = WQ ? R(0.25) * d.Qyzz : R(0);
    const R qC = WQ ? R(0.125) * d.Qxyz : R(0);

    auto ds_of = [&](int i) -> R {
        const int sx = vel(i, 0), sy = vel(i, 1), sz = vel(i, 2);
        const int nzc = (sx != 0) + (sy != 0) + (sz != 0);
        if (nzc == 0) return sRest;
        if (nzc == 1) {
            if (sx) return sF[0] + R(sx) * qF[0];
            if (sy) return sF[1] + R(sy) * qF[1];
            return sF[2] + R(sz) * qF[2];
        }
        if (nzc == 2) {
            if (!sz) return R(sx * sy) * eXY + R(sy) * qXYy + R(sx) * qXYx;
            if (!sy) return R(sx * sz) * eXZ + R(sz) * qXZz + R(sx) * qXZx;
            return R(sy * sz) * eYZ + R(sz) * qYZz + R(sy) * qYZy;
        }
        return R(sx * sy * sz) * qC;
    };
    kbc_gamma_relax<R, GX, DEV>(f, ds_of, fneq_of, iCx, iA9, rho, c, gout, eq_of);
}

// Central-moment variants (section IV; appendix), then kbc_gamma_relax.  The
// shear part is rebuilt from central moments of f - f^eq about the node's u.
// Because f - f^eq carries no mass and no momentum, its second-order central
// moments equal the natural ones, and a third-order one is the natural one
// minus u times second-order ones, e.g. dMt_120 = dM_120 - 2u_y dM_110 -
// u_x dM_020 (raw moments throughout).  The population representation in
// the central basis is the tensor product of one-dimensional inverses: on an
// axis with velocity u the central moments (m0, m1, m2) give
//   f_{-1} = (u^2 - u)/2 m0 + (u - 1/2) m1 + m2/2,
//   f_0    = (1 - u^2) m0 - 2u m1 - m2,
//   f_{+1} = (u^2 + u)/2 m0 + (u + 1/2) m1 + m2/2,
// so ds~ is three separable passes over a 3x3x3 array that holds only the
// 13 second- and third-order entries kept in s.
template <typename R, int V, bool GX, bool DEV, typename FneqFn, typename EqFn>
__host__ __device__ __forceinline__ void kbc_relax_central(R (&f)[27], const DMom<R>& d,
                                                           const R (&u)[3], FneqFn fneq_of,
                                                           const R (&iCx)[3], const R (&iA9)[9],
                                                           double rho, const Coll& c, double* gout,
                                                           EqFn eq_of)
{
    constexpr bool WT = with_t(V);
    constexpr bool WQ = with_q(V);
    R X[3][3][3];
#pragma unroll
    for (int k = 0; k < 27; ++k) X[k % 3][(k / 3) % 3][k / 9] = R(0);
    if constexpr (WT) {
        X[2][0][0] = d.Dxx;
        X[0][2][0] = d.Dyy;
        X[0][0][2] = d.Dzz;
    } else {
        // d~ alone: the deviatoric (trace-free) part of the diagonal
        const R t3 = (d.Dxx + d.Dyy + d.Dzz) * R(1.0 / 3.0);
        X[2][0][0] = d.Dxx - t3;
        X[0][2][0] = d.Dyy - t3;
        X[0][0][2] = d.Dzz - t3;
    }
    X[1][1][0] = d.Pxy;
    X[1][0][1] = d.Pxz;
    X[0][1][1] = d.Pyz;
    if constexpr (WQ) {
        const R ux = u[0], uy = u[1], uz = u[2];
        X[1][2][0] = d.Qxyy - R(2) * uy * d.Pxy - ux * d.Dyy;
        X[1][0][2] = d.Qxzz - R(2) * uz * d.Pxz - ux * d.Dzz;
        X[2][1][0] = d.Qxxy - R(2) * ux * d.Pxy - uy * d.Dxx;
        X[0][1][2] = d.Qyzz - R(2) * uz * d.Pyz - uy * d.Dzz;
        X[2][0][1] = d.Qxxz - R(2) * ux * d.Pxz - uz * d.Dxx;
        X[0][2][1] = d.Qyyz - R(2) * uy * d.Pyz - uz * d.Dyy;
        X[1][1][1] = d.Qxyz - ux * d.Pyz - uy * d.Pxz - uz * d.Pxy;
    }
    // G[a][v+1][p]: weight of the central moment of order p on axis a in the
    // population with velocity v
    R G[3][3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const R ua = u[a], u2 = ua * ua;
        G[a][0][0] = R(0.5) * (u2 - ua);
        G[a][0][1] = ua - R(0.5);
        G[a][0][2] = R(0.5);
        G[a][1][0] = R(1) - u2;
        G[a][1][1] = R(-2) * ua;
        G[a][1][2] = R(-1);
        G[a][2][0] = R(0.5) * (u2 + ua);
        G[a][2][1] = ua + R(0.5);
        G[a][2][2] = R(0.5);
    }
    // z, then y, then x
    R Z1[3][3][3], Z2[3][3][3], ds[27];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int vz = 0; vz < 3; ++vz)
                Z1[p][q][vz] = G[2][vz][0] * X[p][q][0] + G[2][vz][1] * X[p][q][1] +
                               G[2][vz][2] * X[p][q][2];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int vy = 0; vy < 3; ++vy)
#pragma unroll
            for (int vz = 0; vz < 3; ++vz)
                Z2[p][vy][vz] = G[1][vy][0] * Z1[p][0][vz] + G[1][vy][1] * Z1[p][1][vz] +
                                G[1][vy][2] * Z1[p][2][vz];
#pragma unroll
    for (int vx = 0; vx < 3; ++vx)
#pragma unroll
        for (int vy = 0; vy < 3; ++vy)
#pragma unroll
            for (int vz = 0; vz < 3; ++vz)
                ds[vx + 3 * vy + 9 * vz] = G[0][vx][0] * Z2[0][vy][vz] +
                                           G[0][vx][1] * Z2[1][vy][vz] +
                                           G[0][vx][2] * Z2[2][vy][vz];
    kbc_gamma_relax<R, GX, DEV>(f, [&](int i) -> R { return ds[i]; }, fneq_of, iCx, iA9, rho, c,
                                gout, eq_of);
}

// gout, when given, receives the gamma used at this node.
template <int S, int V, bool GX = false>
__host__ __device__ __forceinline__ void collide(typename Traits<S>::R (&f)[27], const Coll& c,
                                                 double* gout = nullptr)
{
    using R = typename Traits<S>::R;
    constexpr bool DEV = Traits<S>::kDev;

    if constexpr (Traits<S>::kMixed) {
        // rho, u and f - f^eq from the deviations g, in FP64
        double X0[9], X1[9];
#pragma unroll
        for (int yz = 0; yz < 9; ++yz) {
            const double fm = f[3 * yz + 0], f0 = f[3 * yz + 1], fp = f[3 * yz + 2];
            X0[yz] = (fm + f0) + fp;
            X1[yz] = fp - fm;
        }
        double drho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
        for (int yz = 0; yz < 9; ++yz) {
            const int vy = yz % 3 - 1, vz = yz / 3 - 1;
            drho += X0[yz];
            jx += X1[yz];
            if (vy) jy += vy * X0[yz];
            if (vz) jz += vz * X0[yz];
        }
        const double rho = 1.0 + drho;
        const double irho = 1.0 / rho;
        const double u[3] = {jx * irho, jy * irho, jz * irho};
        double E[3][3], dE[3][3], dm2;
#pragma unroll
        for (int a = 0; a < 3; ++a) marginals1d<double, true>(u[a], E[a], dE[a], dm2);
        // f_i - f_i^eq = g_i - (rho e_x e_y e_z - W_x W_y W_z), expanded so
        // that no O(1) terms cancel
        R fneq[27];
#pragma unroll
        for (int yz = 0; yz < 9; ++yz) {
            const int ay = yz % 3, az = yz / 3;
            const double A = E[1][ay] * E[2][az];
            const double B = dE[1][ay] * E[2][az] + w1(ay - 1) * dE[2][az];
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                const double C = dE[0][ax] + drho * E[0][ax];
                const double geq = A * C + w1(ax - 1) * B;
                fneq[3 * yz + ax] = (R)((double)f[3 * yz + ax] - geq);
            }
        }
        // in FP32: the moment differences are moments of f - f^eq
        R M[3][3][3];
        moments27<R>(fneq, M);
        DMom<R> d;
        d.T = M[2][0][0] + M[0][2][0] + M[0][0][2];
        d.Nxz = M[2][0][0] - M[0][0][2];
        d.Nyz = M[0][2][0] - M[0][0][2];
        d.Pxy = M[1][1][0];
        d.Pxz = M[1][0][1];
        d.Pyz = M[0][1][1];
        d.Qxyy = M[1][2][0];
        d.Qxzz = M[1][0][2];
        d.Qxxy = M[2][1][0];
        d.Qyzz = M[0][1][2];
        d.Qxxz = M[2][0][1];
        d.Qyyz = M[0][2][1];
        d.Qxyz = M[1][1][1];
        d.Dxx = M[2][0][0];
        d.Dyy = M[0][2][0];
        d.Dzz = M[0][0][2];
        R iE[3][3], Ef[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
#pragma unroll
            for (int k = 0; k < 3; ++k) Ef[a][k] = (R)E[a][k];
            recip3<R>(Ef[a], iE[a]);
        }
        R iA9[9], iCx[3];
#pragma unroll
        for (int yz = 0; yz < 9; ++yz) iA9[yz] = iE[1][yz % 3] * iE[2][yz / 3];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) iCx[ax] = (R)irho * iE[0][ax];
        auto fneq_of = [&](int i) -> R { return fneq[i]; };
        // f^eq - W in FP64, re-formed where the exact stabilizer needs it
        auto eq_of = [&](int i) -> double {
            const int ax = i % 3, ay = (i / 3) % 3, az = i / 9;
            const double A = E[1][ay] * E[2][az];
            const double B = dE[1][ay] * E[2][az] + w1(ay - 1) * dE[2][az];
            const double C = dE[0][ax] + drho * E[0][ax];
            return A * C + w1(ax - 1) * B;
        };
        if constexpr (is_central(V)) {
            const R uf[3] = {(R)u[0], (R)u[1], (R)u[2]};
            kbc_relax_central<R, V, GX, true>(f, d, uf, fneq_of, iCx, iA9, rho, c, gout, eq_of);
        } else {
            kbc_relax<R, V, GX, true>(f, d, fneq_of, iCx, iA9, rho, c, gout, eq_of);
        }
    } else {
        // raw moments R_pqr = sum_i f_i vx^p vy^q vz^r (p,q,r <= 2)
        R M[3][3][3];
        moments27<R>(f, M);
        // rho and u (deviation forms: rho = 1 + sum g, sum v W = 0)
        const R drho = DEV ? M[0][0][0] : M[0][0][0] - R(1);
        const R rho = DEV ? R(1) + drho : M[0][0][0];
        const R irho = rcp_(rho);
        const R u[3] = {M[1][0][0] * irho, M[0][1][0] * irho, M[0][0][1] * irho};

        // one-dimensional equilibrium marginals (Eq. entropic_eq)
        R E[3][3], dE[3][3], dm2[3], m2[3], iE[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            marginals1d<R, DEV>(u[a], E[a], dE[a], dm2[a]);
            m2[a] = R(1.0 / 3.0) + dm2[a];
            recip3<R>(E[a], iE[a]);
        }

        // moment differences; equilibrium moments in closed form:
        // rho m_p(u_x) m_q(u_y) m_r(u_z); the second-order diagonal ones
        // carry the weights' share 1/3 in the deviation forms
        R dD[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const R Mdiag = a == 0 ? M[2][0][0] : (a == 1 ? M[0][2][0] : M[0][0][2]);
            if constexpr (DEV) dD[a] = Mdiag - (drho * R(1.0 / 3.0) + rho * dm2[a]);
            else dD[a] = Mdiag - rho * m2[a];
        }
        DMom<R> d;
        d.T = dD[0] + dD[1] + dD[2];
        d.Nxz = dD[0] - dD[2];
        d.Nyz = dD[1] - dD[2];
        d.Pxy = M[1][1][0] - rho * u[0] * u[1];
        d.Pxz = M[1][0][1] - rho * u[0] * u[2];
        d.Pyz = M[0][1][1] - rho * u[1] * u[2];
        d.Qxyy = M[1][2][0] - rho * u[0] * m2[1];
        d.Qxzz = M[1][0][2] - rho * u[0] * m2[2];
        d.Qxxy = M[2][1][0] - rho * m2[0] * u[1];
        d.Qyzz = M[0][1][2] - rho * u[1] * m2[2];
        d.Qxxz = M[2][0][1] - rho * m2[0] * u[2];
        d.Qyyz = M[0][2][1] - rho * m2[1] * u[2];
        d.Qxyz = M[1][1][1] - rho * u[0] * u[1] * u[2];
        d.Dxx = dD[0];
        d.Dyy = dD[1];
        d.Dzz = dD[2];

        // equilibrium (or its deviation from W) and 1/f^eq, from the marginals
        R A9[9], B9[9], iA9[9];
#pragma unroll
        for (int yz = 0; yz < 9; ++yz) {
            const int ay = yz % 3, az = yz / 3;
            A9[yz] = E[1][ay] * E[2][az];
            iA9[yz] = iE[1][ay] * iE[2][az];
            if constexpr (DEV) B9[yz] = dE[1][ay] * E[2][az] + R(w1(ay - 1)) * dE[2][az];
            else B9[yz] = R(0);
        }
        R Cx[3], iCx[3];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            if constexpr (DEV) Cx[ax] = dE[0][ax] + drho * E[0][ax];
            else Cx[ax] = rho * E[0][ax];
            iCx[ax] = irho * iE[0][ax];
        }
        // f_i - f_i^eq, re-formed in each pass to keep register pressure low
        auto fneq_of = [&](int i) -> R {
            const int ax = i % 3, yz = i / 3;
            if constexpr (DEV) return f[i] - (A9[yz] * Cx[ax] + R(w1(ax - 1)) * B9[yz]);
            else return f[i] - A9[yz] * Cx[ax];
        };
        // the equilibrium in the stored form (f^eq, or f^eq - W)
        auto eq_of = [&](int i) -> double {
            const int ax = i % 3, yz = i / 3;
            if constexpr (DEV) return (double)(A9[yz] * Cx[ax] + R(w1(ax - 1)) * B9[yz]);
            else return (double)(A9[yz] * Cx[ax]);
        };
        if constexpr (is_central(V))
            kbc_relax_central<R, V, GX, DEV>(f, d, u, fneq_of, iCx, iA9, (double)rho, c, gout,
                                             eq_of);
        else
            kbc_relax<R, V, GX, DEV>(f, d, fneq_of, iCx, iA9, (double)rho, c, gout, eq_of);
    }
}

}  // namespace kbc
