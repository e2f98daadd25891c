/*
 * kbc_oracle.h -- plain FP64 CPU reference ("oracle") for the D3Q27 KBC
 * entropic multi-relaxation lattice Boltzmann step of
 * Boesch, Chikatamarla & Karlin, "Entropic multi-relaxation lattice
 * Boltzmann scheme for turbulent flows" (arXiv:1507.02518).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU path.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header, table or helper with
 * the GPU library, and the GPU library never calls it.
 *
 * Conventions (readings where the paper is silent; each is listed with its
 * reason in the design notes of the repository):
 *   - velocity index i = (vx+1) + 3*(vy+1) + 9*(vz+1); rest population i=13;
 *     opposite direction 26-i.  The paper labels velocities only by triads.
 *   - population fields are [27][nz][ny][nx], x fastest, FP64.
 *   - velocity fields are [3][nz][ny][nx].
 *   - the stored state F(t) is the pre-collision field; one step is the
 *     KBC collision of section IV (the mirror state of Eq. ksh-mirror in
 *     Eq. Egeneral) followed by periodic propagation
 *     f_i(x+v_i, t+1) = f'_i(x, t) (Eq. Egeneral).
 *   - variant: 0 -> s=d, 1 -> s=d+t, 2 -> s=d+q, 3 -> s=d+t+q (section IV,
 *     natural moments); 4..7 -> the same four in the central-moment basis,
 *     s = d~, d~+t~, d~+q~, d~+t~+q~ (section IV; appendix).
 *   - gamma mode: 0 -> entropic estimate gamma* (Eq. result21) with the
 *     fallback gamma=2 when <dh|dh> <= gamma_eps*rho (the paper leaves 0/0
 *     undefined); 1 -> fixed gamma = gamma_value; 2 -> exact root of the
 *     entropy-maximum condition (Eq. result1).
 */
#ifndef KBC_ORACLE_H
#define KBC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { KBCO_S_D = 0, KBCO_S_DT = 1, KBCO_S_DQ = 2, KBCO_S_DTQ = 3,
       KBCO_S_CD = 4, KBCO_S_CDT = 5, KBCO_S_CDQ = 6, KBCO_S_CDTQ = 7 };
enum { KBCO_GAMMA_ESTIMATE = 0, KBCO_GAMMA_FIXED = 1, KBCO_GAMMA_EXACT = 2 };

/* Lattice (section II, Eqs. D1Q3, D3Q27vel, weights, sound). */
void   kbco_velocity(int i, int v[3]);
double kbco_weight(int i);
double kbco_beta_from_nu(double nu);             /* Eq. viscosity solved for beta */

/* Product-form entropic equilibrium (section II, Eq. entropic_eq). */
void   kbco_feq(double rho, const double u[3], double feq[27]);

/* Natural moments M_pqr, p,q,r in {0,1,2} (section III, Eq. natmoments):
 * M[p + 3q + 9r] = sum_i f_i vx^p vy^q vz^r / rho. Returns rho. */
double kbco_natural_moments(const double f[27], double M[27]);

/* Populations from natural moments (section III, Eq. moment_rep). */
void   kbco_f_from_moments(double rho, const double M[27], double f[27]);

/* The kinematic part k and the parts d, t, q of table s_parts (section IV),
 * evaluated from natural moments M and density rho. */
void   kbco_parts(double rho, const double M[27], double k[27], double d[27],
                  double t[27], double q[27]);

/* Shear part s for a variant (section IV): d, d+t, d+q or d+t+q. */
void   kbco_s_part(double rho, const double M[27], int variant, double s[27]);

/* Central moments rho Mt_pqr = sum_i f_i (v_ix-u_x)^p (v_iy-u_y)^q (v_iz-u_z)^r,
 * u = j/rho (section III, central basis): Mt[p + 3q + 9r].  Returns rho;
 * writes u to u_out unless it is NULL. */
double kbco_central_moments(const double f[27], double Mt[27], double u_out[3]);

/* Parts k~, d~, t~, q~ of the population representation in the central basis
 * (appendix, Eqs. cmf000-cmfxyz) from rho, u and the central moments Mt.
 * Any output may be NULL. */
void   kbco_central_parts(double rho, const double u[3], const double Mt[27],
                          double k[27], double d[27], double t[27], double q[27]);

/* Weight of the central moment Mt_m (m = p + 3q + 9r) in f_i / rho at
 * velocity u: one column of the inverse of the central-moment map. */
void   kbco_central_column(const double u[3], int m, double col[27]);

/* Shear part s of f for any variant 0..7. */
void   kbco_s_of(const double f[27], int variant, double s[27]);

/* One node: the KBC collision of section IV.  rho and u of F; f^eq (Eq.
 * entropic_eq); ds = s - s^eq and dh = f - f^eq - ds (Eqs.
 * ksh-representation, ksh-mirror; table s_parts); gamma (Eq. result21, or
 * Eq. result1, or fixed); P = F - beta (2 ds + gamma dh) (Eq. Egeneral with
 * the mirror state of Eq. ksh-mirror).  Every output pointer except P may be
 * NULL.  Returns the gamma used. */
double kbco_collide(const double F[27], double beta, int variant,
                    int gamma_mode, double gamma_value, double gamma_eps,
                    double P[27], double feq[27], double ds[27], double dh[27]);

/* Exact stabilizer: the root in gamma of Eq. result1 (section IV), on the
 * interval where every post-collision population stays positive.
 * Returns NAN if no bracketing interval exists. */
double kbco_gamma_exact(const double feq[27], const double ds[27],
                        const double dh[27], double beta);

/* Whole-lattice operations on [27][nz][ny][nx] fields. */
void kbco_init_feq(int64_t nx, int64_t ny, int64_t nz, const double* u,
                   const double* rho /* NULL -> 1 */, double* F);
void kbco_collide_field(int64_t nx, int64_t ny, int64_t nz, double beta,
                        int variant, int gamma_mode, double gamma_value,
                        double gamma_eps, const double* F, double* P,
                        double* gamma_field /* NULL allowed */);
void kbco_stream(int64_t nx, int64_t ny, int64_t nz, const double* P, double* Fnext);
/* collide then stream; P is caller scratch of the same size as F */
void kbco_step(int64_t nx, int64_t ny, int64_t nz, double beta, int variant,
               int gamma_mode, double gamma_value, double gamma_eps,
               const double* F, double* P, double* Fnext);

/* Diagnostics (section V). */
void   kbco_macros(int64_t nx, int64_t ny, int64_t nz, const double* F,
                   double* rho /* NULL allowed */, double* u /* NULL allowed */);
double kbco_energy(int64_t nx, int64_t ny, int64_t nz, const double* u);
double kbco_enstrophy(int64_t nx, int64_t ny, int64_t nz, const double* u);

int kbco_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
