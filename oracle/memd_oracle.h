/*
 * memd_oracle.h -- plain FP64 CPU oracle for the MEMD lattice update with a
 * spatially varying permittivity (Fahrenberger & Holm, arXiv:1309.7859).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this code: only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no source with the HIP library.
 *
 * Conventions (every array is FP64, owned by the caller):
 *   lattice    L x L x L periodic, spacing a, site v = i + L*(j + L*k), x fastest
 *   link field X[3*Ns], component d at X[d*Ns + v]: link from v to v + e_d
 *   plaquette  Y[3*Ns], component d at Y[d*Ns + v]: corner v, spanned by e_d1, e_d2
 *              where (d, d1, d2) is a cyclic permutation of (x, y, z)
 *   positions  r[3*n] unfolded, xyz interleaved per ion; charges q[n]
 *   units      rationalised, eps0 = 1: a^2 * sum_d [D_d(v) - D_d(v - e_d)] = q_v
 */
#ifndef MEMD_ORACLE_H
#define MEMD_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

int orc_version(void);
/* OpenMP threads the stencil loops use, and a way to set them (n > 0). */
int orc_threads(void);
void orc_set_threads(int n);

/* Linear (cloud-in-cell) charge assignment to the 8 corners of the cell
 * (section "Self energy interaction"; section "Error estimates"). */
void orc_spread(int L, double a, int n, const double *q, const double *r, double *rho);

/* Site -> link permittivity (Fig. 2b; eq. dielectric-interpolation).
 * Returns the number of interface links (ratio above r_thr, harmonic mean). */
int orc_eps_site_to_link(int L, const double *eps_site, double r_thr, double *eps_link);

/* eta = 1/eps per link, directional harmonic means eps_h[3] and the cell
 * permittivity eps_cell[Ns] (harmonic mean over the 12 edges of each cell). */
void orc_eps_derived(int L, const double *eps_link, double *eta, double eps_h[3],
                     double *eps_cell);

/* Salt-dependent permittivity per link: eps = eps_w - slope * c_link with the
 * CIC ion density smoothed by the periodic 3x3x3 vertex box mean. */
void orc_salt_eps(int L, double a, int n, const double *r, double eps_w, double slope,
                  double eps_floor, double *eps_link);

/* Discrete curl C (links -> plaquettes) and its adjoint C^T (plaquettes -> links). */
void orc_curl(int L, double a, const double *X, double *Y);
void orc_curl_adj(int L, double a, const double *Y, double *X);
/* Lattice divergence of a link field, (div X)(v) = sum_d [X_d(v) - X_d(v-e_d)] / a. */
void orc_div(int L, double a, const double *X, double *out);

/* Initial solution of Gauss's law by the plane -> line -> vertex recursion
 * (Fig. 1 and the equations beside it), written on D. */
void orc_recursion(int L, double a, const double *rho, double *D);
/* Add a constant per direction so that mean_v D_d = -P_d / V. */
void orc_mean_shift(int L, double a, const double P[3], double *D);
/* Relaxation to curl E = 0 by minimising 1/2 a^3 sum eta D^2 over D + C^T theta
 * (conjugate gradients, Jacobi preconditioner).  Returns 0 on convergence, 1
 * otherwise.  res_out = a*max|C(eta D)| / max|eta D|. */
int orc_relax(int L, double a, const double *eta, double *D, double tol, int max_iter,
              int *iters_out, double *res_out);
/* Relative curl measure used by orc_relax. */
double orc_curl_measure(int L, double a, const double *eta, const double *D);

/* Leapfrog halves: B -= dt C(eta D) (Faraday), D += dt c^2 C^T B (Ampere). */
void orc_faraday(int L, double a, double dt, const double *eta, const double *D, double *B);
void orc_ampere(int L, double a, double dt, double c, const double *B, double *D);
/* Move every ion by disp (dimension split x, y, z) and deposit its current
 * into D so that Gauss's law is kept; r is updated in place. */
void orc_deposit(int L, double a, int n, const double *q, double *r, const double *disp,
                 double *D);
/* One full step: Faraday, Ampere, deposit. */
void orc_step(int L, double a, double dt, double c, const double *eta, int n,
              const double *q, double *r, const double *disp, double *D, double *B);

/* Observables */
void orc_gauss_residual(int L, double a, const double *D, const double *rho,
                        double *max_abs, double *rms);
void orc_dipole(int n, const double *q, const double *r, double P[3]);
/* Periodic lattice Green's function with the k = 0 mode removed, at the
 * offsets (0,0,0), (1,0,0), (1,1,0), (1,1,1). */
void orc_greens(int L, double G[4]);
/* Cell self-energy sum S(f) = sum_{v,v'} w_v w_v' G(v - v') and dS/df. */
void orc_self_sum(const double G[4], const double f[3], double *S, double dS[3]);
/* Corrected forces F[3n] and per-ion self energies Uself[n] (may be NULL);
 * scheme 0 subtracts the Green's-function self force, 1 the direct one. */
void orc_forces(int L, double a, int n, const double *q, const double *r, const double *D,
                const double *eta, const double *eps_cell, const double eps_h[3],
                const double G[4], const double P[3], int scheme, double *F, double *Uself);
/* Energies: out = {W_E, W_B (shadow), U_self, U_dip, E_corrected}. */
void orc_energy(int L, double a, double dt, double c, const double *eta, const double *D,
                const double *B, double U_self, const double P[3], const double eps_h[3],
                double out[5]);

/* Philox4x32-10 counter-based generator and the seeded Gaussian displacement
 * stream built on it (ion i, step t). */
void orc_philox4x32_10(const unsigned int ctr[4], const unsigned int key[2], unsigned int out[4]);
void orc_seeded_displacements(unsigned long long seed, int t, int n, double sigma, double *out);

#ifdef __cplusplus
}
#endif
#endif
