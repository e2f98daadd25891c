/*
 * kbc_oracle.c -- plain FP64 CPU reference ("oracle") for the D3Q27 KBC
 * lattice Boltzmann step of Boesch, Chikatamarla & Karlin,
 * "Entropic multi-relaxation lattice Boltzmann scheme for turbulent flows"
 * (arXiv:1507.02518).
 *
 * TEST INFRASTRUCTURE ONLY: this file is the oracle the GPU library is tested against.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load it; the GPU library never does, and the two share no code.
 *
 * Everything here is written for the eye, not for speed: each step of the
 * paper is evaluated in the paper's order and notation with plain loops and
 * IEEE double arithmetic (libm sqrt/log).  Nodes are independent within a
 * collision, so the only parallelism is an OpenMP loop over z-planes, which
 * does not change any result.
 */
#include "kbc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Lattice: section II.                                                      */
/* ------------------------------------------------------------------------ */

/* D3Q27 velocities as the tensor product of three copies of the D1Q3 set
 * {-1, 0, 1} (Eqs. D1Q3 and D3Q27vel).  Index i = (vx+1) + 3(vy+1) + 9(vz+1). */
void kbco_velocity(int i, int v[3])
{
    v[0] = i % 3 - 1;
    v[1] = (i / 3) % 3 - 1;
    v[2] = i / 9 - 1;
}

/* One-dimensional weights W_0 = 2/3, W_{+-1} = 1/6 (section II, below
 * Eq. sound), and their product over the three axes (Eq. weights). */
static double weight_1d(int c)
{
    return c == 0 ? 2.0 / 3.0 : 1.0 / 6.0;
}

double kbco_weight(int i)
{
    int v[3];
    kbco_velocity(i, v);
    return weight_1d(v[0]) * weight_1d(v[1]) * weight_1d(v[2]);
}

/* Kinematic viscosity nu = c_s^2 (1/(2 beta) - 1/2) (Eq. viscosity) with
 * c_s^2 = 1/3 (Eq. sound), solved for beta. */
double kbco_beta_from_nu(double nu)
{
    const double cs2 = 1.0 / 3.0;
    return 1.0 / (2.0 * (nu / cs2 + 0.5));
}

/* ------------------------------------------------------------------------ */
/* Equilibrium: section II, Eq. entropic_eq.                                 */
/* ------------------------------------------------------------------------ */

static double eq_A(double u) { return 2.0 - sqrt(1.0 + 3.0 * u * u); }
static double eq_B(double u) { return (2.0 * u + sqrt(1.0 + 3.0 * u * u)) / (1.0 - u); }

/* [B(u)]^v for v in {-1, 0, 1}. */
static double eq_B_pow(double u, int v)
{
    if (v == 0) return 1.0;
    if (v == 1) return eq_B(u);
    return 1.0 / eq_B(u);
}

/* f_i^eq = rho W_i Psi(u) B(u_x)^{v_ix} B(u_y)^{v_iy} B(u_z)^{v_iz},
 * Psi(u) = A(u_x) A(u_y) A(u_z). */
void kbco_feq(double rho, const double u[3], double feq[27])
{
    const double psi = eq_A(u[0]) * eq_A(u[1]) * eq_A(u[2]);
    for (int i = 0; i < 27; ++i) {
        int v[3];
        kbco_velocity(i, v);
        feq[i] = rho * kbco_weight(i) * psi
               * eq_B_pow(u[0], v[0]) * eq_B_pow(u[1], v[1]) * eq_B_pow(u[2], v[2]);
    }
}

/* ------------------------------------------------------------------------ */
/* Moments: section III.                                                     */
/* ------------------------------------------------------------------------ */

static double ipow(int v, int p)
{
    double r = 1.0;
    for (int k = 0; k < p; ++k) r *= (double)v;
    return r;
}

/* rho M_pqr = sum_i f_i vx^p vy^q vz^r (Eq. natmoments), p,q,r in {0,1,2}. */
double kbco_natural_moments(const double f[27], double M[27])
{
    double rho = 0.0;
    for (int i = 0; i < 27; ++i) rho += f[i];
    for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q)
            for (int p = 0; p < 3; ++p) {
                double sum = 0.0;
                for (int i = 0; i < 27; ++i) {
                    int v[3];
                    kbco_velocity(i, v);
                    sum += f[i] * ipow(v[0], p) * ipow(v[1], q) * ipow(v[2], r);
                }
                M[p + 3 * q + 9 * r] = sum / rho;
            }
    return rho;
}

#define MOM(p, q, r) M[(p) + 3 * (q) + 9 * (r)]

/* The named moments of section III.  The paper's list of third-order names
 * repeats Q_yyz and omits Q_xyy and Q_yzz; they are read as Q_xyy = M_120 and
 * Q_yzz = M_012, the only assignment under which the moment representation
 * (Eq. moment_rep) is the inverse of Eq. natmoments. */
typedef struct {
    double ux, uy, uz;
    double T, Nxz, Nyz;
    double Pxy, Pxz, Pyz;
    double Qxyy, Qxzz, Qxxy, Qyzz, Qxxz, Qyyz, Qxyz;
} named_moments;

static named_moments name_moments(const double M[27])
{
    named_moments n;
    n.ux = MOM(1, 0, 0);
    n.uy = MOM(0, 1, 0);
    n.uz = MOM(0, 0, 1);
    n.T = MOM(2, 0, 0) + MOM(0, 2, 0) + MOM(0, 0, 2);
    n.Nxz = MOM(2, 0, 0) - MOM(0, 0, 2);
    n.Nyz = MOM(0, 2, 0) - MOM(0, 0, 2);
    n.Pxy = MOM(1, 1, 0);
    n.Pxz = MOM(1, 0, 1);
    n.Pyz = MOM(0, 1, 1);
    n.Qxyy = MOM(1, 2, 0);
    n.Qxzz = MOM(1, 0, 2);
    n.Qxxy = MOM(2, 1, 0);
    n.Qyzz = MOM(0, 1, 2);
    n.Qxxz = MOM(2, 0, 1);
    n.Qyyz = MOM(0, 2, 1);
    n.Qxyz = MOM(1, 1, 1);
    return n;
}

/* Populations written in the basis of natural moments (Eq. moment_rep).  The
 * direction labels (sigma, lambda, delta) are the signs of the non-zero
 * velocity components; the paper's text calls the third sign gamma, its
 * equations call it delta. */
void kbco_f_from_moments(double rho, const double M[27], double f[27])
{
    const named_moments n = name_moments(M);
    const double M022 = MOM(0, 2, 2), M202 = MOM(2, 0, 2), M220 = MOM(2, 2, 0);
    const double M222 = MOM(2, 2, 2);
    const double M122 = MOM(1, 2, 2), M212 = MOM(2, 1, 2), M221 = MOM(2, 2, 1);
    const double M112 = MOM(1, 1, 2), M121 = MOM(1, 2, 1), M211 = MOM(2, 1, 1);
    for (int i = 0; i < 27; ++i) {
        int v[3];
        kbco_velocity(i, v);
        const double s = v[0], l = v[1], d = v[2];
        const int nz = (v[0] != 0) + (v[1] != 0) + (v[2] != 0);
        double val;
        if (nz == 0) {
            val = rho * (1.0 - n.T + M022 + M202 + M220 - M222);
        } else if (nz == 1 && v[0] != 0) {
            val = rho / 6.0 * (3.0 * s * n.ux + 2.0 * n.Nxz - n.Nyz + n.T
                               - 3.0 * s * n.Qxyy - 3.0 * s * n.Qxzz + 3.0 * s * M122
                               - 3.0 * M202 - 3.0 * M220 + 3.0 * M222);
        } else if (nz == 1 && v[1] != 0) {
            val = rho / 6.0 * (3.0 * l * n.uy - n.Nxz + 2.0 * n.Nyz + n.T
                               - 3.0 * l * n.Qxxy - 3.0 * l * n.Qyzz + 3.0 * l * M212
                               - 3.0 * M022 - 3.0 * M220 + 3.0 * M222);
        } else if (nz == 1) {
            val = rho / 6.0 * (3.0 * d * n.uz - n.Nxz - n.Nyz + n.T
                               - 3.0 * d * n.Qxxz - 3.0 * d * n.Qyyz + 3.0 * d * M221
                               - 3.0 * M022 - 3.0 * M202 + 3.0 * M222);
        } else if (nz == 2 && v[2] == 0) {
            val = rho / 4.0 * (s * l * n.Pxy + l * n.Qxxy + s * n.Qxyy + M220
                               - s * M122 - l * M212 - s * l * M112 - M222);
        } else if (nz == 2 && v[1] == 0) {
            val = rho / 4.0 * (s * d * n.Pxz + d * n.Qxxz + s * n.Qxzz + M202
                               - s * M122 - d * M221 - s * d * M121 - M222);
        } else if (nz == 2) {
            val = rho / 4.0 * (l * d * n.Pyz + d * n.Qyyz + l * n.Qyzz + M022
                               - l * M212 - d * M221 - l * d * M211 - M222);
        } else {
            val = rho / 8.0 * (s * l * d * n.Qxyz + s * M122 + l * M212 + d * M221
                               + s * l * M112 + s * d * M121 + l * d * M211 + M222);
        }
        f[i] = val;
    }
}

/* ------------------------------------------------------------------------ */
/* k / d / t / q parts: section IV, table s_parts.                           */
/* ------------------------------------------------------------------------ */

/* Each entry of the table is a part divided by rho, written in the natural
 * moments; the parts themselves are rho times the entry. */
void kbco_parts(double rho, const double M[27], double k[27], double d[27],
                double t[27], double q[27])
{
    const named_moments n = name_moments(M);
    for (int i = 0; i < 27; ++i) {
        int v[3];
        kbco_velocity(i, v);
        const double s = v[0], l = v[1], dl = v[2];
        double kk = 0.0, dd = 0.0, tt = 0.0, qq = 0.0;
        const int nz = (v[0] != 0) + (v[1] != 0) + (v[2] != 0);
        if (nz == 0) {                                 /* (0,0,0) */
            kk = 1.0;
            tt = -n.T;
        } else if (nz == 1 && v[0] != 0) {             /* (sigma,0,0) */
            kk = s * n.ux / 2.0;
            dd = (2.0 * n.Nxz - n.Nyz) / 6.0;
            tt = n.T / 6.0;
            qq = -s * (n.Qxyy + n.Qxzz) / 2.0;
        } else if (nz == 1 && v[1] != 0) {             /* (0,lambda,0) */
            kk = l * n.uy / 2.0;
            dd = (-n.Nxz + 2.0 * n.Nyz) / 6.0;
            tt = n.T / 6.0;
            qq = -l * (n.Qxxy + n.Qyzz) / 2.0;
        } else if (nz == 1) {                          /* (0,0,delta) */
            kk = dl * n.uz / 2.0;
            dd = (-n.Nxz - n.Nyz) / 6.0;
            tt = n.T / 6.0;
            qq = -dl * (n.Qxxz + n.Qyyz) / 2.0;
        } else if (nz == 2 && v[2] == 0) {             /* (sigma,lambda,0) */
            dd = s * l * n.Pxy / 4.0;
            qq = (l * n.Qxxy + s * n.Qxyy) / 4.0;
        } else if (nz == 2 && v[1] == 0) {             /* (sigma,0,delta) */
            dd = s * dl * n.Pxz / 4.0;
            qq = (dl * n.Qxxz + s * n.Qxzz) / 4.0;
        } else if (nz == 2) {                          /* (0,lambda,delta) */
            dd = l * dl * n.Pyz / 4.0;
            qq = (dl * n.Qyyz + l * n.Qyzz) / 4.0;
        } else {                                       /* (sigma,lambda,delta) */
            qq = s * l * dl * n.Qxyz / 8.0;
        }
        if (k) k[i] = rho * kk;
        if (d) d[i] = rho * dd;
        if (t) t[i] = rho * tt;
        if (q) q[i] = rho * qq;
    }
}

/* s in {d, d+t, d+q, d+t+q}: the four natural-moment KBC models (section IV). */
void kbco_s_part(double rho, const double M[27], int variant, double s[27])
{
    double d[27], t[27], q[27];
    kbco_parts(rho, M, NULL, d, t, q);
    const int with_t = (variant == KBCO_S_DT || variant == KBCO_S_DTQ);
    const int with_q = (variant == KBCO_S_DQ || variant == KBCO_S_DTQ);
    for (int i = 0; i < 27; ++i)
        s[i] = d[i] + (with_t ? t[i] : 0.0) + (with_q ? q[i] : 0.0);
}

/* ------------------------------------------------------------------------ */
/* Central moments (section III, central basis; appendix).                  */
/* ------------------------------------------------------------------------ */

/* rho Mt_pqr = sum_i f_i (vx-ux)^p (vy-uy)^q (vz-uz)^r with u = j/rho. */
double kbco_central_moments(const double f[27], double Mt[27], double u_out[3])
{
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 27; ++i) {
        int v[3];
        kbco_velocity(i, v);
        rho += f[i];
        for (int a = 0; a < 3; ++a) j[a] += v[a] * f[i];
    }
    const double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
    for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q)
            for (int p = 0; p < 3; ++p) {
                double sum = 0.0;
                for (int i = 0; i < 27; ++i) {
                    int v[3];
                    kbco_velocity(i, v);
                    sum += f[i] * pow(v[0] - u[0], p) * pow(v[1] - u[1], q) * pow(v[2] - u[2], r);
                }
                Mt[p + 3 * q + 9 * r] = sum / rho;
            }
    if (u_out) memcpy(u_out, u, sizeof u);
    return rho;
}

/* Inverse of the 27x27 map from populations to central moments at velocity
 * u, C[m][i] = prod_a (v_ia - u_a)^{p_a(m)}, by Gauss-Jordan elimination with
 * partial pivoting.  Cinv[i][m] is the weight of Mt_m in f_i / rho: the
 * population representation in the central basis that the appendix
 * writes out (Eqs. cmf000 to cmfxyz). */
static void central_inverse(const double u[3], double Cinv[27][27])
{
    double A[27][54];
    for (int m = 0; m < 27; ++m) {
        const int p = m % 3, q = (m / 3) % 3, r = m / 9;
        for (int i = 0; i < 27; ++i) {
            int v[3];
            kbco_velocity(i, v);
            A[m][i] = pow(v[0] - u[0], p) * pow(v[1] - u[1], q) * pow(v[2] - u[2], r);
        }
        for (int k = 0; k < 27; ++k) A[m][27 + k] = (k == m) ? 1.0 : 0.0;
    }
    for (int c = 0; c < 27; ++c) {
        int piv = c;
        for (int rr = c + 1; rr < 27; ++rr)
            if (fabs(A[rr][c]) > fabs(A[piv][c])) piv = rr;
        if (piv != c)
            for (int k = 0; k < 54; ++k) {
                const double tmp = A[c][k];
                A[c][k] = A[piv][k];
                A[piv][k] = tmp;
            }
        const double d = A[c][c];
        for (int k = 0; k < 54; ++k) A[c][k] /= d;
        for (int rr = 0; rr < 27; ++rr) {
            if (rr == c || A[rr][c] == 0.0) continue;
            const double fct = A[rr][c];
            for (int k = 0; k < 54; ++k) A[rr][k] -= fct * A[c][k];
        }
    }
    /* A's right half is C^{-1}: rows indexed by the population i */
    for (int i = 0; i < 27; ++i)
        for (int m = 0; m < 27; ++m) Cinv[i][m] = A[i][27 + m];
}

#define CM(p, q, r) ((p) + 3 * (q) + 9 * (r))

/* The parts k~, d~, t~, q~ of the central representation: each collects the
 * terms of Eqs. cmf000-cmfxyz that carry the central moments it names.  k~
 * holds the terms of rho and u alone; d~ those of Pi~_xy, Pi~_xz, Pi~_yz,
 * N~_xz, N~_yz; t~ that of T~; q~ those of the seven Q~.  The normal stress
 * differences and the trace enter through N~_xz = Mt_200 - Mt_002,
 * N~_yz = Mt_020 - Mt_002, T~ = Mt_200 + Mt_020 + Mt_002 (section III). */
void kbco_central_parts(double rho, const double u[3], const double Mt[27], double k[27],
                        double d[27], double t[27], double q[27])
{
    double Ci[27][27];
    central_inverse(u, Ci);
    const double Tt = Mt[CM(2, 0, 0)] + Mt[CM(0, 2, 0)] + Mt[CM(0, 0, 2)];
    const double Nxz = Mt[CM(2, 0, 0)] - Mt[CM(0, 0, 2)];
    const double Nyz = Mt[CM(0, 2, 0)] - Mt[CM(0, 0, 2)];
    for (int i = 0; i < 27; ++i) {
        const double c200 = Ci[i][CM(2, 0, 0)], c020 = Ci[i][CM(0, 2, 0)],
                     c002 = Ci[i][CM(0, 0, 2)];
        /* weights of N~_xz, N~_yz and T~ once Mt_200, Mt_020, Mt_002 are
         * written through them */
        const double wNxz = (2.0 * c200 - c020 - c002) / 3.0;
        const double wNyz = (-c200 + 2.0 * c020 - c002) / 3.0;
        const double wT = (c200 + c020 + c002) / 3.0;
        if (k)
            k[i] = rho * (Ci[i][CM(0, 0, 0)] * Mt[CM(0, 0, 0)] + Ci[i][CM(1, 0, 0)] * Mt[CM(1, 0, 0)] +
                          Ci[i][CM(0, 1, 0)] * Mt[CM(0, 1, 0)] + Ci[i][CM(0, 0, 1)] * Mt[CM(0, 0, 1)]);
        if (d)
            d[i] = rho * (Ci[i][CM(1, 1, 0)] * Mt[CM(1, 1, 0)] + Ci[i][CM(1, 0, 1)] * Mt[CM(1, 0, 1)] +
                          Ci[i][CM(0, 1, 1)] * Mt[CM(0, 1, 1)] + wNxz * Nxz + wNyz * Nyz);
        if (t) t[i] = rho * wT * Tt;
        if (q)
            q[i] = rho * (Ci[i][CM(1, 2, 0)] * Mt[CM(1, 2, 0)] + Ci[i][CM(1, 0, 2)] * Mt[CM(1, 0, 2)] +
                          Ci[i][CM(2, 1, 0)] * Mt[CM(2, 1, 0)] + Ci[i][CM(0, 1, 2)] * Mt[CM(0, 1, 2)] +
                          Ci[i][CM(2, 0, 1)] * Mt[CM(2, 0, 1)] + Ci[i][CM(0, 2, 1)] * Mt[CM(0, 2, 1)] +
                          Ci[i][CM(1, 1, 1)] * Mt[CM(1, 1, 1)]);
    }
}

/* Column of the central representation: the weight of Mt_m in f_i / rho. */
void kbco_central_column(const double u[3], int m, double col[27])
{
    double Ci[27][27];
    central_inverse(u, Ci);
    for (int i = 0; i < 27; ++i) col[i] = Ci[i][m];
}

/* s evaluated on an arbitrary population vector g: natural-moment parts
 * (table s_parts) for variants 0-3, central-moment parts for 4-7. */
static void s_of(const double g[27], int variant, double s[27])
{
    if (variant >= KBCO_S_CD) {
        double Mt[27], u[3], d[27], t[27], q[27];
        const double rho = kbco_central_moments(g, Mt, u);
        kbco_central_parts(rho, u, Mt, NULL, d, t, q);
        const int with_t = (variant == KBCO_S_CDT || variant == KBCO_S_CDTQ);
        const int with_q = (variant == KBCO_S_CDQ || variant == KBCO_S_CDTQ);
        for (int i = 0; i < 27; ++i)
            s[i] = d[i] + (with_t ? t[i] : 0.0) + (with_q ? q[i] : 0.0);
        return;
    }
    double M[27];
    const double rho = kbco_natural_moments(g, M);
    kbco_s_part(rho, M, variant, s);
}

/* Shear part of f for any variant (natural or central basis). */
void kbco_s_of(const double f[27], int variant, double s[27]) { s_of(f, variant, s); }

/* ------------------------------------------------------------------------ */
/* Stabilizer: section IV, Eqs. result1 and result21.                        */
/* ------------------------------------------------------------------------ */

/* Left side of Eq. result1 as a function of gamma. */
static double result1_lhs(const double feq[27], const double ds[27],
                          const double dh[27], double beta, double gamma)
{
    double sum = 0.0;
    for (int i = 0; i < 27; ++i)
        sum += dh[i] * log(1.0 + ((1.0 - beta * gamma) * dh[i]
                                  - (2.0 * beta - 1.0) * ds[i]) / feq[i]);
    return sum;
}

/* The argument of every logarithm in Eq. result1 is f'_i / f_i^eq; it is
 * positive on an open interval of gamma, on which the left side falls
 * monotonically from +inf to -inf.  The root is found by bisection. */
double kbco_gamma_exact(const double feq[27], const double ds[27],
                        const double dh[27], double beta)
{
    double lo = -INFINITY, hi = INFINITY;
    for (int i = 0; i < 27; ++i) {
        const double x = feq[i] + dh[i] - (2.0 * beta - 1.0) * ds[i];
        if (dh[i] > 0.0) {
            const double b = x / (beta * dh[i]);
            if (b < hi) hi = b;
        } else if (dh[i] < 0.0) {
            const double b = x / (beta * dh[i]);
            if (b > lo) lo = b;
        }
    }
    if (!(lo < hi) || isinf(lo) || isinf(hi)) return NAN;
    for (int it = 0; it < 400; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        const double g = result1_lhs(feq, ds, dh, beta, mid);
        if (g > 0.0) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* ------------------------------------------------------------------------ */
/* Collision of section IV: the KBC mirror state inserted in Eq. Egeneral.  */
/* ------------------------------------------------------------------------ */

/* Conserved fields of f (section I, with Eq. S): rho = sum_i f_i and
 * rho u = sum_i v_i f_i.  Returns rho. */
static double conserved_fields(const double f[27], double u[3])
{
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 27; ++i) {
        int v[3];
        kbco_velocity(i, v);
        rho += f[i];
        j[0] += v[0] * f[i];
        j[1] += v[1] * f[i];
        j[2] += v[2] * f[i];
    }
    u[0] = j[0] / rho;
    u[1] = j[1] / rho;
    u[2] = j[2] / rho;
    return rho;
}

/* Eq. ksh-representation splits every population as f = k + s + h, and
 * Eq. ksh-mirror uses the same parts evaluated at equilibrium.  The shear
 * part s is read from table s_parts (natural moments) or from the central
 * basis, on f and on f^eq separately: ds = s - s^eq.  The kinematic part k
 * depends only on rho and u, which f and f^eq share, so it cancels and the
 * higher-order difference is what is left: dh = h - h^eq = f - f^eq - ds. */
static void part_differences(const double f[27], const double feq[27], int variant,
                             double ds[27], double dh[27])
{
    double s[27], seq[27];
    s_of(f, variant, s);
    s_of(feq, variant, seq);
    for (int i = 0; i < 27; ++i) {
        ds[i] = s[i] - seq[i];
        dh[i] = f[i] - feq[i] - ds[i];
    }
}

/* The stabilizer gamma of the mirror state.  Eq. result21: the estimate
 * gamma = 1/beta - (2 - 1/beta) <ds|dh> / <dh|dh> in the entropic scalar
 * product <X|Y> = sum_i X_i Y_i / f_i^eq; or the root of Eq. result1; or a
 * fixed value.  Where <dh|dh> <= gamma_eps rho (at equilibrium both
 * products vanish and the estimate is 0/0) gamma is the LBGK value 2. */
static double stabilizer(const double feq[27], const double ds[27], const double dh[27],
                         double rho, double beta, int gamma_mode, double gamma_value,
                         double gamma_eps)
{
    if (gamma_mode == KBCO_GAMMA_FIXED) return gamma_value;
    double sh = 0.0, hh = 0.0;
    for (int i = 0; i < 27; ++i) {
        sh += ds[i] * dh[i] / feq[i];
        hh += dh[i] * dh[i] / feq[i];
    }
    if (hh <= gamma_eps * rho) return 2.0;
    if (gamma_mode == KBCO_GAMMA_EXACT) {
        const double g = kbco_gamma_exact(feq, ds, dh, beta);
        return isnan(g) ? 2.0 : g;
    }
    return 1.0 / beta - (2.0 - 1.0 / beta) * sh / hh;
}

/* Eq. Egeneral relaxes f toward the mirror state, f' = f + beta (f^mirr - f).
 * With the mirror state of Eq. ksh-mirror, f^mirr - f = 2 (s^eq - s) +
 * gamma (h^eq - h) = -(2 ds + gamma dh), so f' = f - beta (2 ds + gamma dh). */
static void relax(const double f[27], const double ds[27], const double dh[27], double beta,
                  double gamma, double P[27])
{
    for (int i = 0; i < 27; ++i) P[i] = f[i] - beta * (2.0 * ds[i] + gamma * dh[i]);
}

double kbco_collide(const double F[27], double beta, int variant,
                    int gamma_mode, double gamma_value, double gamma_eps,
                    double P[27], double feq_out[27], double ds_out[27],
                    double dh_out[27])
{
    double u[3], feq[27], ds[27], dh[27];
    const double rho = conserved_fields(F, u);
    kbco_feq(rho, u, feq);                              /* Eq. entropic_eq */
    part_differences(F, feq, variant, ds, dh);
    const double gamma = stabilizer(feq, ds, dh, rho, beta, gamma_mode, gamma_value, gamma_eps);
    relax(F, ds, dh, beta, gamma, P);
    if (feq_out) memcpy(feq_out, feq, sizeof feq);
    if (ds_out) memcpy(ds_out, ds, sizeof ds);
    if (dh_out) memcpy(dh_out, dh, sizeof dh);
    return gamma;
}

/* ------------------------------------------------------------------------ */
/* Whole lattice.                                                            */
/* ------------------------------------------------------------------------ */

static int64_t wrap(int64_t a, int64_t n)
{
    const int64_t r = a % n;
    return r < 0 ? r + n : r;
}

void kbco_init_feq(int64_t nx, int64_t ny, int64_t nz, const double* u,
                   const double* rho, double* F)
{
    const int64_t nn = nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                const int64_t n = (z * ny + y) * nx + x;
                const double un[3] = {u[n], u[nn + n], u[2 * nn + n]};
                double feq[27];
                kbco_feq(rho ? rho[n] : 1.0, un, feq);
                for (int i = 0; i < 27; ++i) F[i * nn + n] = feq[i];
            }
}

void kbco_collide_field(int64_t nx, int64_t ny, int64_t nz, double beta,
                        int variant, int gamma_mode, double gamma_value,
                        double gamma_eps, const double* F, double* P,
                        double* gamma_field)
{
    const int64_t nn = nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                const int64_t n = (z * ny + y) * nx + x;
                double fn[27], pn[27];
                for (int i = 0; i < 27; ++i) fn[i] = F[i * nn + n];
                const double g = kbco_collide(fn, beta, variant, gamma_mode,
                                              gamma_value, gamma_eps, pn,
                                              NULL, NULL, NULL);
                for (int i = 0; i < 27; ++i) P[i * nn + n] = pn[i];
                if (gamma_field) gamma_field[n] = g;
            }
}

/* Propagation: f_i(x + v_i, t+1) = f'_i(x, t) on the periodic box
 * (Eq. Egeneral), i.e. F_i(x) = P_i(x - v_i). */
void kbco_stream(int64_t nx, int64_t ny, int64_t nz, const double* P, double* Fnext)
{
    const int64_t nn = nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                const int64_t n = (z * ny + y) * nx + x;
                for (int i = 0; i < 27; ++i) {
                    int v[3];
                    kbco_velocity(i, v);
                    const int64_t sx = wrap(x - v[0], nx);
                    const int64_t sy = wrap(y - v[1], ny);
                    const int64_t sz = wrap(z - v[2], nz);
                    Fnext[i * nn + n] = P[i * nn + (sz * ny + sy) * nx + sx];
                }
            }
}

void kbco_step(int64_t nx, int64_t ny, int64_t nz, double beta, int variant,
               int gamma_mode, double gamma_value, double gamma_eps,
               const double* F, double* P, double* Fnext)
{
    kbco_collide_field(nx, ny, nz, beta, variant, gamma_mode, gamma_value,
                       gamma_eps, F, P, NULL);
    kbco_stream(nx, ny, nz, P, Fnext);
}

/* ------------------------------------------------------------------------ */
/* Diagnostics: section V.                                                   */
/* ------------------------------------------------------------------------ */

void kbco_macros(int64_t nx, int64_t ny, int64_t nz, const double* F,
                 double* rho, double* u)
{
    const int64_t nn = nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < nn; ++n) {
        double r = 0.0, j[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < 27; ++i) {
            int v[3];
            kbco_velocity(i, v);
            const double f = F[i * nn + n];
            r += f;
            j[0] += v[0] * f;
            j[1] += v[1] * f;
            j[2] += v[2] * f;
        }
        if (rho) rho[n] = r;
        if (u) {
            u[n] = j[0] / r;
            u[nn + n] = j[1] / r;
            u[2 * nn + n] = j[2] / r;
        }
    }
}

static void mean_velocity(int64_t nn, const double* u, double ubar[3])
{
    for (int a = 0; a < 3; ++a) {
        double s = 0.0;
        for (int64_t n = 0; n < nn; ++n) s += u[a * nn + n];
        ubar[a] = s / (double)nn;
    }
}

/* k = (1/2) < u'_a u'_a >, u' = u - <u>, <.> the mean over the nodes. */
double kbco_energy(int64_t nx, int64_t ny, int64_t nz, const double* u)
{
    const int64_t nn = nx * ny * nz;
    double ubar[3];
    mean_velocity(nn, u, ubar);
    double s = 0.0;
    for (int64_t n = 0; n < nn; ++n)
        for (int a = 0; a < 3; ++a) {
            const double up = u[a * nn + n] - ubar[a];
            s += up * up;
        }
    return 0.5 * s / (double)nn;
}

/* Omega = (1/2) < |curl u'|^2 >, derivatives by second-order central
 * differences on the periodic grid (the in-run choice of section V.A). */
double kbco_enstrophy(int64_t nx, int64_t ny, int64_t nz, const double* u)
{
    const int64_t nn = nx * ny * nz;
    double ubar[3];
    mean_velocity(nn, u, ubar);
    double s = 0.0;
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                const int64_t xp = wrap(x + 1, nx), xm = wrap(x - 1, nx);
                const int64_t yp = wrap(y + 1, ny), ym = wrap(y - 1, ny);
                const int64_t zp = wrap(z + 1, nz), zm = wrap(z - 1, nz);
#define UP(a, X, Y, Z) (u[(a) * nn + ((Z) * ny + (Y)) * nx + (X)] - ubar[a])
                const double duz_dy = 0.5 * (UP(2, x, yp, z) - UP(2, x, ym, z));
                const double duy_dz = 0.5 * (UP(1, x, y, zp) - UP(1, x, y, zm));
                const double dux_dz = 0.5 * (UP(0, x, y, zp) - UP(0, x, y, zm));
                const double duz_dx = 0.5 * (UP(2, xp, y, z) - UP(2, xm, y, z));
                const double duy_dx = 0.5 * (UP(1, xp, y, z) - UP(1, xm, y, z));
                const double dux_dy = 0.5 * (UP(0, x, yp, z) - UP(0, x, ym, z));
#undef UP
                const double wx = duz_dy - duy_dz;
                const double wy = dux_dz - duz_dx;
                const double wz = duy_dx - dux_dy;
                s += wx * wx + wy * wy + wz * wz;
            }
    return 0.5 * s / (double)nn;
}

int kbco_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
