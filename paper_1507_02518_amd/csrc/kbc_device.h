// kbc_device.h -- device-side definitions of the D3Q27 KBC update for gfx950:
// lattice constants, index helpers, kernel parameter blocks, storage codecs
// and the per-node collision of section IV of Boesch, Chikatamarla & Karlin
// (arXiv:1507.02518).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kbc {

enum Storage : int { ST_F64 = 0, ST_F32 = 1, ST_F16 = 2 };
enum Variant : int { V_D = 0, V_DT = 1, V_DQ = 2, V_DTQ = 3 };
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

// Geometry of one periodic box inside a population buffer.
struct Geom {
    uint32_t nx, ny, nz, nnodes;   // nnodes = nx*ny*nz
    FastDiv dnx, dny;
    uint64_t plane;                // elements between consecutive directions
};

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

struct StepParams {
    const void* src;
    void* dst;
    Geom g;
    Coll c;
    float scale[27];      // FP16 storage: stored = (f - W) * scale
    float inv_scale[27];
};

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
};
template <> struct Traits<ST_F32> {
    using T = float;
    using R = float;
    static constexpr bool kDev = true;
};
template <> struct Traits<ST_F16> {
    using T = _Float16;
    using R = float;
    static constexpr bool kDev = true;
};

template <int S>
__device__ __forceinline__ typename Traits<S>::R decode(typename Traits<S>::T v, float inv_scale)
{
    if constexpr (S == ST_F16) return (float)v * inv_scale;
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
// the deviation forms).  Steps follow the listing at the end of section IV:
//  1. rho, u from a separable 3x3x3 moment transform of f;
//  2. f^eq from its one-dimensional marginals: with S = sqrt(1+3u^2) the
//     product-form factors of section II reduce to e_0 = (4 - 2S)/3,
//     e_{+-1} = ((2S - 1)/3 +- u)/2 per axis, f_i^eq = rho e(vx) e(vy) e(vz);
//  3-4. ds from the differences of the 13 second- and third-order natural
//     moments of f and f^eq (table s_parts); the equilibrium moments factor
//     as rho m_p(u_x) m_q(u_y) m_r(u_z), m_0 = 1, m_1 = u, m_2 = (2S - 1)/3;
//  5. dh = f - f^eq - ds;
//  6. gamma = 1/beta - (2 - 1/beta) <ds|dh>/<dh|dh>, 1/f^eq_i separable;
//     gamma = 2 where <dh|dh> <= gamma_eps * rho (0/0 at equilibrium);
//  7. f' = f - beta (2 ds + gamma dh).
// ---------------------------------------------------------------------------
template <int S, int V>
__host__ __device__ __forceinline__ void collide(typename Traits<S>::R (&f)[27], const Coll& c)
{
    using R = typename Traits<S>::R;
    constexpr bool DEV = Traits<S>::kDev;
    constexpr bool WT = (V == V_DT || V == V_DTQ);
    constexpr bool WQ = (V == V_DQ || V == V_DTQ);
    const R third = R(1.0 / 3.0);

    // --- 1. raw moments R_pqr = sum_i f_i vx^p vy^q vz^r (p,q,r <= 2) ------
    R X[3][9];
#pragma unroll
    for (int yz = 0; yz < 9; ++yz) {
        const R fm = f[3 * yz + 0], f0 = f[3 * yz + 1], fp = f[3 * yz + 2];
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
    R M[3][3][3];
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

    // rho and u (deviation forms: rho = 1 + sum g, sum v W = 0)
    const R drho = DEV ? M[0][0][0] : M[0][0][0] - R(1);
    const R rho = DEV ? R(1) + drho : M[0][0][0];
    const R irho = R(1) / rho;
    const R u[3] = {M[1][0][0] * irho, M[0][1][0] * irho, M[0][0][1] * irho};

    // --- 2. one-dimensional equilibrium marginals --------------------------
    R E[3][3], dE[3][3], m2[3], dm2[3], iE[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const R ua = u[a];
        const R q3 = R(3) * ua * ua;
        const R Sq = sqrt(R(1) + q3);
        R sm1;  // S - 1, formed without cancellation in the FP32 forms
        if constexpr (DEV) sm1 = q3 / (R(1) + Sq);
        else sm1 = Sq - R(1);
        dm2[a] = R(2.0 / 3.0) * sm1;
        m2[a] = third + dm2[a];
        const R half_u = R(0.5) * ua;
        dE[a][1] = -dm2[a];
        dE[a][2] = R(0.5) * dm2[a] + half_u;
        dE[a][0] = R(0.5) * dm2[a] - half_u;
        E[a][1] = R(2.0 / 3.0) + dE[a][1];
        E[a][2] = R(1.0 / 6.0) + dE[a][2];
        E[a][0] = R(1.0 / 6.0) + dE[a][0];
        // three reciprocals from one division
        const R pm = E[a][0] * E[a][2];
        const R ip = R(1) / (pm * E[a][1]);
        iE[a][1] = pm * ip;
        iE[a][2] = E[a][1] * E[a][0] * ip;
        iE[a][0] = E[a][1] * E[a][2] * ip;
    }

    // --- 3-4. moment differences and the shear part per direction class ----
    // second-order diagonal moments carry the weights' share 1/3 (deviation
    // forms) and rho m_2 = (1 + drho)(1/3 + dm_2)
    R dD[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const R Mdiag = a == 0 ? M[2][0][0] : (a == 1 ? M[0][2][0] : M[0][0][2]);
        if constexpr (DEV) dD[a] = Mdiag - (drho * third + rho * dm2[a]);
        else dD[a] = Mdiag - rho * m2[a];
    }
    const R dT = dD[0] + dD[1] + dD[2];
    const R dNxz = dD[0] - dD[2];
    const R dNyz = dD[1] - dD[2];
    const R dPxy = M[1][1][0] - rho * u[0] * u[1];
    const R dPxz = M[1][0][1] - rho * u[0] * u[2];
    const R dPyz = M[0][1][1] - rho * u[1] * u[2];
    const R dQxyy = M[1][2][0] - rho * u[0] * m2[1];
    const R dQxzz = M[1][0][2] - rho * u[0] * m2[2];
    const R dQxxy = M[2][1][0] - rho * m2[0] * u[1];
    const R dQyzz = M[0][1][2] - rho * u[1] * m2[2];
    const R dQxxz = M[2][0][1] - rho * m2[0] * u[2];
    const R dQyyz = M[0][2][1] - rho * m2[1] * u[2];
    const R dQxyz = M[1][1][1] - rho * u[0] * u[1] * u[2];

    const R t6 = WT ? dT * R(1.0 / 6.0) : R(0);
    const R sRest = WT ? -dT : R(0);
    const R sF[3] = {(R(2) * dNxz - dNyz) * R(1.0 / 6.0) + t6,
                     (R(2) * dNyz - dNxz) * R(1.0 / 6.0) + t6,
                     -(dNxz + dNyz) * R(1.0 / 6.0) + t6};
    const R qF[3] = {WQ ? R(-0.5) * (dQxyy + dQxzz) : R(0),
                     WQ ? R(-0.5) * (dQxxy + dQyzz) : R(0),
                     WQ ? R(-0.5) * (dQxxz + dQyyz) : R(0)};
    const R eXY = R(0.25) * dPxy, eXZ = R(0.25) * dPxz, eYZ = R(0.25) * dPyz;
    const R qXYy = WQ ? R(0.25) * dQxxy : R(0), qXYx = WQ ? R(0.25) * dQxyy : R(0);
    const R qXZz = WQ ? R(0.25) * dQxxz : R(0), qXZx = WQ ? R(0.25) * dQxzz : R(0);
    const R qYZz = WQ ? R(0.25) * dQyyz : R(0), qYZy = WQ ? R(0.25) * dQyzz : R(0);
    const R qC = WQ ? R(0.125) * dQxyz : R(0);

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
    // f_i - f_i^eq
    auto fneq_of = [&](int i) -> R {
        const int ax = i % 3, yz = i / 3;
        if constexpr (DEV) return f[i] - (A9[yz] * Cx[ax] + R(w1(ax - 1)) * B9[yz]);
        else return f[i] - A9[yz] * Cx[ax];
    };

    // --- 5-6. dh and the entropic scalar products --------------------------
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
        gamma = (hhd <= c.gamma_eps * (double)rho) ? R(2) : R(c.inv_beta - c.c2 * shd / hhd);
    }

    // --- 7. relax: f' = f - beta (2 ds + gamma dh) -------------------------
    const R beta = R(c.beta);
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        const R ds = ds_of(i);
        const R dh = fneq_of(i) - ds;
        f[i] = f[i] - beta * (R(2) * ds + gamma * dh);
    }
}

}  // namespace kbc
