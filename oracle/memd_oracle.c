/*
 * memd_oracle.c -- plain, slow, FP64 CPU oracle for the MEMD lattice update
 * with a spatially varying permittivity (Fahrenberger & Holm, arXiv:1309.7859).
 *
 * TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the product path.  Each function
 * follows the passage of the paper it cites, in the paper's order, without
 * blocking or fusion.  Where the paper is silent or garbled the reading taken
 * is stated next to the code.  OpenMP is used only on loops whose iterations
 * write disjoint elements (results do not depend on the thread count);
 * every reduction and every scatter is serial, in index order.
 */
#include "memd_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

int orc_version(void) { return 1; }

#ifdef _OPENMP
#include <omp.h>
int orc_threads(void) { return omp_get_max_threads(); }
void orc_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
#else
int orc_threads(void) { return 1; }
void orc_set_threads(int n) { (void)n; }
#endif

/* ------------------------------------------------------------------ lattice */

static long wrapi(long i, int L) {
    long m = i % L;
    return m < 0 ? m + L : m;
}

static size_t site(int L, long i, long j, long k) {
    return (size_t)wrapi(i, L) + (size_t)L * ((size_t)wrapi(j, L) + (size_t)L * (size_t)wrapi(k, L));
}

/* site index of (i,j,k) + s * e_d */
static size_t shifted(int L, long i, long j, long k, int d, long s) {
    long x[3] = {i, j, k};
    x[d] += s;
    return site(L, x[0], x[1], x[2]);
}

/* Fold one unfolded coordinate: t = u/a, cell k = floor(t), fraction f = t - k
 * in [0,1), folded cell index c = k mod L. */
static void fold(double u, double a, int L, long *kcell, long *c, double *f) {
    double t = u / a;
    double fl = floor(t);
    *f = t - fl;
    *kcell = (long)fl;
    *c = wrapi((long)fl, L);
}

/* Linear interpolation weights: w(0; f) = 1 - f, w(1; f) = f. */
static double wgt(int o, double f) { return o ? f : 1.0 - f; }

/* ------------------------------------------------------------- charge (CIC) */

/* Linear charge interpolation onto the 8 corners of the ion's cell
 * (section "Self energy interaction", the linear-order requirement; section
 * "Error estimates", the one-cell cutoff). */
void orc_spread(int L, double a, int n, const double *q, const double *r, double *rho) {
    size_t Ns = (size_t)L * L * L;
    memset(rho, 0, Ns * sizeof(double));
    for (int i = 0; i < n; ++i) {
        long kc[3], c[3];
        double f[3];
        for (int d = 0; d < 3; ++d) fold(r[3 * i + d], a, L, &kc[d], &c[d], &f[d]);
        for (int oz = 0; oz < 2; ++oz)
            for (int oy = 0; oy < 2; ++oy)
                for (int ox = 0; ox < 2; ++ox) {
                    double w = wgt(ox, f[0]) * wgt(oy, f[1]) * wgt(oz, f[2]);
                    rho[site(L, c[0] + ox, c[1] + oy, c[2] + oz)] += q[i] * w;
                }
    }
}

/* ------------------------------------------------------------- permittivity */

/* Fig. 2b and eq. dielectric-interpolation: the link between sites v and
 * v + e_d takes the mean of the two site values; where the two values differ
 * strongly the link is an interface link and takes the harmonic (series)
 * combination.  Reading: "differ strongly" means max/min > r_thr, and with
 * only site values known the interface sits halfway (d1 = d2 = a/2), so
 * 1/eps = (1/2)/eps1 + (1/2)/eps2. */
int orc_eps_site_to_link(int L, const double *eps_site, double r_thr, double *eps_link) {
    size_t Ns = (size_t)L * L * L;
    int n_interface = 0;
    for (long k = 0; k < L; ++k)
        for (long j = 0; j < L; ++j)
            for (long i = 0; i < L; ++i) {
                size_t v = site(L, i, j, k);
                for (int d = 0; d < 3; ++d) {
                    double e1 = eps_site[v];
                    double e2 = eps_site[shifted(L, i, j, k, d, 1)];
                    double hi = e1 > e2 ? e1 : e2, lo = e1 > e2 ? e2 : e1;
                    double e;
                    if (hi / lo > r_thr) {
                        e = 1.0 / (0.5 / e1 + 0.5 / e2);
                        ++n_interface;
                    } else {
                        e = 0.5 * (e1 + e2);
                    }
                    eps_link[(size_t)d * Ns + v] = e;
                }
            }
    return n_interface;
}

/* eta = 1/eps per link; eps_h[d] = harmonic mean over all d-links (the exact
 * stiffness of a uniform D_d mode, used by the dipole correction); eps_cell =
 * harmonic mean over the 12 edges of the cell (the "eps constant within the
 * cell" assumption of the Green's-function self-energy correction). */
void orc_eps_derived(int L, const double *eps_link, double *eta, double eps_h[3],
                     double *eps_cell) {
    size_t Ns = (size_t)L * L * L;
    for (size_t x = 0; x < 3 * Ns; ++x) eta[x] = 1.0 / eps_link[x];
    for (int d = 0; d < 3; ++d) {
        double s = 0.0;
        for (size_t v = 0; v < Ns; ++v) s += eta[(size_t)d * Ns + v];
        eps_h[d] = (double)Ns / s;
    }
    if (!eps_cell) return;
    for (long k = 0; k < L; ++k)
        for (long j = 0; j < L; ++j)
            for (long i = 0; i < L; ++i) {
                double s = 0.0;
                for (int d = 0; d < 3; ++d) {
                    int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
                    for (int o2 = 0; o2 < 2; ++o2)
                        for (int o1 = 0; o1 < 2; ++o1) {
                            long x[3] = {i, j, k};
                            x[d1] += o1;
                            x[d2] += o2;
                            s += eta[(size_t)d * Ns + site(L, x[0], x[1], x[2])];
                        }
                }
                eps_cell[site(L, i, j, k)] = 12.0 / s;
            }
}

/* Salt-dependent permittivity (the introduction's motivation: eps of water
 * falls as the salt concentration rises).  n_v = CIC ion count per a^3,
 * nbar = periodic 3x3x3 box mean, link concentration = mean of its two ends,
 * eps = eps_w - slope * c, floored at eps_floor. */
void orc_salt_eps(int L, double a, int n, const double *r, double eps_w, double slope,
                  double eps_floor, double *eps_link) {
    size_t Ns = (size_t)L * L * L;
    double *ones = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double *cnt = (double *)malloc(Ns * sizeof(double));
    double *nbar = (double *)malloc(Ns * sizeof(double));
    for (int i = 0; i < n; ++i) ones[i] = 1.0;
    orc_spread(L, a, n, ones, r, cnt);
    double inv_cell = 1.0 / (a * a * a);
    for (long k = 0; k < L; ++k)
        for (long j = 0; j < L; ++j)
            for (long i = 0; i < L; ++i) {
                double s = 0.0;
                for (int dz = -1; dz <= 1; ++dz)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dx = -1; dx <= 1; ++dx)
                            s += cnt[site(L, i + dx, j + dy, k + dz)] * inv_cell;
                nbar[site(L, i, j, k)] = s / 27.0;
            }
    for (long k = 0; k < L; ++k)
        for (long j = 0; j < L; ++j)
            for (long i = 0; i < L; ++i) {
                size_t v = site(L, i, j, k);
                for (int d = 0; d < 3; ++d) {
                    double cl = 0.5 * (nbar[v] + nbar[shifted(L, i, j, k, d, 1)]);
                    double e = eps_w - slope * cl;
                    eps_link[(size_t)d * Ns + v] = e < eps_floor ? eps_floor : e;
                }
            }
    free(ones);
    free(cnt);
    free(nbar);
}

/* --------------------------------------------------------- discrete operators */

/* Same finite-difference curl as the original algorithm (section "Extension of
 * the algorithm", discretisation paragraph):
 *   (C X)_d(v) = [X_d2(v+e_d1) - X_d2(v) - X_d1(v+e_d2) + X_d1(v)] / a        */
void orc_curl(int L, double a, const double *X, double *Y) {
    size_t Ns = (size_t)L * L * L;
#pragma omp parallel for schedule(static)
    for (long k = 0; k < L; ++k)
        for (long j = 0; j < L; ++j)
            for (long i = 0; i < L; ++i) {
                size_t v = site(L, i, j, k);
                for (int d = 0; d < 3; ++d) {
                    int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
                    double t = X[(size_t)d2 * Ns + shifted(L, i, j, k, d1, 1)] - X[(size_t)d2 * Ns + v] -
                               X[(size_t)d1 * Ns + shifted(L, i, j, k, d2, 1)] + X[(size_t)d1 * Ns + v];
                    Y[(size_t)d * Ns + v] = t / a;
                }
            }
}

/* Adjoint of C under the plain sum inner product:
 *   (C^T Y)_d(v) = [Y_d2(v) - Y_d2(v-e_d1) - Y_d1(v) + Y_d1(v-e_d2)] / a        */
void orc_curl_adj(int L, double a, const double *Y, double *X) {
    size_t Ns = (size_t)L * L * L;
#pragma omp parallel for schedule(static)
    for (long k = 0; k < L; ++k)
        for (long j = 0; j < L; ++j)
            for (long i = 0; i < L; ++i) {
                size_t v = site(L, i, j, k);
                for (int d = 0; d < 3; ++d) {
                    int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
                    double t = Y[(size_t)d2 * Ns + v] - Y[(size_t)d2 * Ns + shifted(L, i, j, k, d1, -1)] -
                               Y[(size_t)d1 * Ns + v] + Y[(size_t)d1 * Ns + shifted(L, i, j, k, d2, -1)];
                    X[(size_t)d * Ns + v] = t / a;
                }
            }
}

void orc_div(int L, double a, const double *X, double *out) {
    size_t Ns = (size_t)L * L * L;
#pragma omp parallel for schedule(static)
    for (long k = 0; k < L; ++k)
        for (long j = 0; j < L; ++j)
            for (long i = 0; i < L; ++i) {
                size_t v = site(L, i, j, k);
                double s = 0.0;
                for (int d = 0; d < 3; ++d)
                    s += X[(size_t)d * Ns + v] - X[(size_t)d * Ns + shifted(L, i, j, k, d, -1)];
                out[v] = s / a;
            }
}

/* ------------------------------------------------------------ initial solve */

/* Initial solution of Gauss's law (Fig. 1 caption and the equations beside
 * it).  Reading: the recursion is run on D (so eps plays no part here; it
 * enters in the relaxation), q_plane is the per-vertex average of the plane
 * (total / L^2), the order is z planes, then y lines within each plane, then
 * single vertices along x, and each stage adds the running sum of the averages
 * (divided by a^2) to the links of that stage and subtracts the average from
 * the vertices.  Gauss's law then holds by telescoping; each plane and each
 * line is neutral after its subtraction, which closes the periodic sums. */
void orc_recursion(int L, double a, const double *rho, double *D) {
    size_t Ns = (size_t)L * L * L;
    double a2 = a * a;
    double *rem = (double *)malloc(Ns * sizeof(double));
    memcpy(rem, rho, Ns * sizeof(double));
    double *Dx = D, *Dy = D + Ns, *Dz = D + 2 * Ns;

    double run = 0.0;
    for (long k = 0; k < L; ++k) {
        double Q = 0.0;
        for (long j = 0; j < L; ++j)
            for (long i = 0; i < L; ++i) Q += rem[site(L, i, j, k)];
        double qplane = Q / ((double)L * L);
        run += qplane;
        for (long j = 0; j < L; ++j)
            for (long i = 0; i < L; ++i) {
                Dz[site(L, i, j, k)] = run / a2;
                rem[site(L, i, j, k)] -= qplane;
            }
    }
    for (long k = 0; k < L; ++k) {
        double runy = 0.0;
        for (long j = 0; j < L; ++j) {
            double Q = 0.0;
            for (long i = 0; i < L; ++i) Q += rem[site(L, i, j, k)];
            double qline = Q / (double)L;
            runy += qline;
            for (long i = 0; i < L; ++i) {
                Dy[site(L, i, j, k)] = runy / a2;
                rem[site(L, i, j, k)] -= qline;
            }
        }
    }
    for (long k = 0; k < L; ++k)
        for (long j = 0; j < L; ++j) {
            double runx = 0.0;
            for (long i = 0; i < L; ++i) {
                runx += rem[site(L, i, j, k)];
                Dx[site(L, i, j, k)] = runx / a2;
            }
        }
    free(rem);
}

/* Section "Periodicity": the periodic lattice ties the uniform (k = 0) part of
 * D to the dipole moment of the unfolded coordinates.  Reading: start from
 * mean_v D_d = -P_d / V, the value every current update then preserves. */
void orc_mean_shift(int L, double a, const double P[3], double *D) {
    size_t Ns = (size_t)L * L * L;
    double V = pow((double)L * a, 3);
    for (int d = 0; d < 3; ++d) {
        double s = 0.0;
        for (size_t v = 0; v < Ns; ++v) s += D[(size_t)d * Ns + v];
        double shift = -P[d] / V - s / (double)Ns;
        for (size_t v = 0; v < Ns; ++v) D[(size_t)d * Ns + v] += shift;
    }
}

static double maxabs(const double *x, size_t m) {
    double s = 0.0;
    for (size_t t = 0; t < m; ++t) {
        double y = fabs(x[t]);
        if (y > s) s = y;
    }
    return s;
}

static double dotp(const double *x, const double *y, size_t m) {
    double s = 0.0;
    for (size_t t = 0; t < m; ++t) s += x[t] * y[t];
    return s;
}

double orc_curl_measure(int L, double a, const double *eta, const double *D) {
    size_t M = 3 * (size_t)L * L * L;
    double *X = (double *)malloc(M * sizeof(double));
    double *Y = (double *)malloc(M * sizeof(double));
    for (size_t t = 0; t < M; ++t) X[t] = eta[t] * D[t];
    orc_curl(L, a, X, Y);
    double num = a * maxabs(Y, M), den = maxabs(X, M);
    free(X);
    free(Y);
    return den > 0.0 ? num / den : num;
}

/* The relaxation step after the recursion: minimising the field energy at
 * fixed charges is equivalent to curl E = 0 (section "Extension of the
 * algorithm", after the recursion).  Reading: minimise W = 1/2 a^3 sum eta D^2
 * over D + C^T theta, which keeps div D (div C^T = 0) and the mean of D (the
 * mean of C^T theta is 0).  The normal equations C eta C^T theta = -C eta D are
 * solved by conjugate gradients with a Jacobi preconditioner; D is updated in
 * place of theta.  The true residual replaces the recursive one every 5
 * iterations and whenever the recursive one passes the test; the system is
 * singular, so iterating past convergence is never done. */
int orc_relax(int L, double a, const double *eta, double *D, double tol, int max_iter,
              int *iters_out, double *res_out) {
    size_t Ns = (size_t)L * L * L, M = 3 * Ns;
    double *X = (double *)malloc(M * sizeof(double));
    double *r = (double *)malloc(M * sizeof(double));
    double *z = (double *)malloc(M * sizeof(double));
    double *p = (double *)malloc(M * sizeof(double));
    double *w = (double *)malloc(M * sizeof(double));
    double *qv = (double *)malloc(M * sizeof(double));
    double *dinv = (double *)malloc(M * sizeof(double));
    double a2 = a * a;

    /* diagonal of C eta C^T: the 4 links of each plaquette, each with weight 1/a^2 */
    for (long k = 0; k < L; ++k)
        for (long j = 0; j < L; ++j)
            for (long i = 0; i < L; ++i) {
                size_t v = site(L, i, j, k);
                for (int d = 0; d < 3; ++d) {
                    int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
                    double s = eta[(size_t)d2 * Ns + shifted(L, i, j, k, d1, 1)] + eta[(size_t)d2 * Ns + v] +
                               eta[(size_t)d1 * Ns + shifted(L, i, j, k, d2, 1)] + eta[(size_t)d1 * Ns + v];
                    dinv[(size_t)d * Ns + v] = a2 / s;
                }
            }

    int it = 0, converged = 0, replace = 1, stalls = 0;
    double res = 0.0, rz = 0.0, den = 0.0, best = HUGE_VAL;
    double *Dbest = (double *)malloc(M * sizeof(double));
    for (;;) {
        if (replace) {
            /* residual replacement: r = -C(eta D) from D itself, and the test */
            for (size_t t = 0; t < M; ++t) X[t] = eta[t] * D[t];
            orc_curl(L, a, X, r);
            for (size_t t = 0; t < M; ++t) r[t] = -r[t];
            den = maxabs(X, M);
            res = den > 0.0 ? a * maxabs(r, M) / den : 0.0;
            if (res <= tol) {
                converged = 1;
                break;
            }
            if (res < best) {
                best = res;
                memcpy(Dbest, D, M * sizeof(double));
            }
            /* below the attainable accuracy the iteration drifts: keep the best */
            if (it >= max_iter || stalls >= 3 || res > 1e3 * best) {
                memcpy(D, Dbest, M * sizeof(double));
                res = best;
                break;
            }
            for (size_t t = 0; t < M; ++t) z[t] = dinv[t] * r[t];
            rz = dotp(r, z, M);
            if (it == 0) memcpy(p, z, M * sizeof(double));
            replace = 0;
        }
        orc_curl_adj(L, a, p, w);
        for (size_t t = 0; t < M; ++t) X[t] = eta[t] * w[t];
        orc_curl(L, a, X, qv);
        double pq = dotp(p, qv, M);
        ++it;
        if (!(pq > 0.0)) {
            /* the direction fell into the null space of C eta C^T: restart */
            memcpy(p, z, M * sizeof(double));
            replace = 1;
            ++stalls;
            continue;
        }
        double alpha = rz / pq;
        for (size_t t = 0; t < M; ++t) {
            D[t] += alpha * w[t];
            r[t] -= alpha * qv[t];
        }
        for (size_t t = 0; t < M; ++t) z[t] = dinv[t] * r[t];
        double rz_new = dotp(r, z, M);
        double beta = rz_new / rz;
        rz = rz_new;
        for (size_t t = 0; t < M; ++t) p[t] = z[t] + beta * p[t];
        /* the recursive residual says "converged": confirm with the true one;
         * a refusal means the recursion has drifted (count it as a stall) */
        if (a * maxabs(r, M) <= tol * den) {
            replace = 1;
            ++stalls;
        } else if (it % 5 == 0) {
            replace = 1;
        }
    }
    if (iters_out) *iters_out = it;
    if (res_out) *res_out = res;
    free(X);
    free(r);
    free(z);
    free(p);
    free(w);
    free(qv);
    free(dinv);
    free(Dbest);
    return converged ? 0 : 1;
}

/* ----------------------------------------------------------------- dynamics */

/* Faraday's law with E = D/eps (eq. faraday, eq. bfield).  Reading: the printed
 * "-curl D" drops the permittivity; with dA/dt = -D/eps (eq. DandA) and
 * B = curl A the update is dB/dt = -curl(D/eps). */
void orc_faraday(int L, double a, double dt, const double *eta, const double *D, double *B) {
    size_t M = 3 * (size_t)L * L * L;
    double *X = (double *)malloc(M * sizeof(double));
    double *Y = (double *)malloc(M * sizeof(double));
    for (size_t t = 0; t < M; ++t) X[t] = eta[t] * D[t];
    orc_curl(L, a, X, Y);
    for (size_t t = 0; t < M; ++t) B[t] -= dt * Y[t];
    free(X);
    free(Y);
}

/* Ampere's law without the current term (eq. ampere, eq. dfield); the current
 * enters through orc_deposit. */
void orc_ampere(int L, double a, double dt, double c, const double *B, double *D) {
    size_t M = 3 * (size_t)L * L * L;
    double *X = (double *)malloc(M * sizeof(double));
    orc_curl_adj(L, a, B, X);
    for (size_t t = 0; t < M; ++t) D[t] += dt * c * c * X[t];
    free(X);
}

/* Particle motion enters as currents on links (eq. constraint: dD/dt + j = curl
 * dTheta/dt), keeping Gauss's law exact.  Reading: the move of each ion is split
 * by dimension, x then y then z, each axis moved with the others held at their
 * current values; along the moving axis the path is cut at cell faces, and each
 * piece [u_a, u_b] inside cell k carries the current q (u_b - u_a)/a onto the 4
 * d-links of that cell with the transverse linear weights, i.e. D_d on those
 * links decreases by q (u_b - u_a)/a * w(o1; f_d1) w(o2; f_d2) / a^2.  Ions are
 * processed in index order. */
void orc_deposit(int L, double a, int n, const double *q, double *r, const double *disp,
                 double *D) {
    size_t Ns = (size_t)L * L * L;
    double a2 = a * a;
    for (int i = 0; i < n; ++i) {
        for (int d = 0; d < 3; ++d) {
            int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
            long k1, c1, k2, c2;
            double f1, f2;
            fold(r[3 * i + d1], a, L, &k1, &c1, &f1);
            fold(r[3 * i + d2], a, L, &k2, &c2, &f2);
            double u0 = r[3 * i + d];
            double u1 = u0 + disp[3 * i + d];
            if (u1 != u0) {
                double lo = u0 < u1 ? u0 : u1, hi = u0 < u1 ? u1 : u0;
                double sgn = u1 > u0 ? 1.0 : -1.0;
                long klo = (long)floor(lo / a), khi = (long)floor(hi / a);
                for (long kc = klo; kc <= khi; ++kc) {
                    double s0 = (double)kc * a, s1 = (double)(kc + 1) * a;
                    double sa = lo > s0 ? lo : s0;
                    double sb = hi < s1 ? hi : s1;
                    double len = sb - sa;
                    if (!(len > 0.0)) continue;
                    double amount = q[i] * sgn * (len / a) / a2;
                    for (int o2 = 0; o2 < 2; ++o2)
                        for (int o1 = 0; o1 < 2; ++o1) {
                            long x[3];
                            x[d] = kc;
                            x[d1] = c1 + o1;
                            x[d2] = c2 + o2;
                            D[(size_t)d * Ns + site(L, x[0], x[1], x[2])] -=
                                amount * wgt(o1, f1) * wgt(o2, f2);
                        }
                }
            }
            r[3 * i + d] = u1;
        }
    }
}

/* Order of one step (reading of the leapfrog, B at half-integer times):
 * B^{n+1/2} = B^{n-1/2} - dt C(eta D^n); D* = D^n + dt c^2 C^T B^{n+1/2};
 * then the ions move and their currents are deposited into D*. */
void orc_step(int L, double a, double dt, double c, const double *eta, int n,
              const double *q, double *r, const double *disp, double *D, double *B) {
    orc_faraday(L, a, dt, eta, D, B);
    orc_ampere(L, a, dt, c, B, D);
    orc_deposit(L, a, n, q, r, disp, D);
}

/* -------------------------------------------------------------- observables */

void orc_gauss_residual(int L, double a, const double *D, const double *rho,
                        double *max_abs, double *rms) {
    size_t Ns = (size_t)L * L * L;
    double *dv = (double *)malloc(Ns * sizeof(double));
    orc_div(L, a, D, dv);
    double m = 0.0, s = 0.0;
    for (size_t v = 0; v < Ns; ++v) {
        double R = a * a * a * dv[v] - rho[v];
        if (fabs(R) > m) m = fabs(R);
        s += R * R;
    }
    *max_abs = m;
    *rms = sqrt(s / (double)Ns);
    free(dv);
}

/* Total dipole moment of the unfolded coordinates (section "Periodicity"). */
void orc_dipole(int n, const double *q, const double *r, double P[3]) {
    P[0] = P[1] = P[2] = 0.0;
    for (int i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) P[d] += q[i] * r[3 * i + d];
}

/* Lattice Green's function (eq. greens and the Brillouin-zone integral that
 * follows it) on the periodic L^3 lattice, where the integral becomes a sum
 * over the L^3 wave vectors k = 2 pi m / L; the k = 0 term is dropped (the
 * neutralising background of a periodic system):
 *   G(n) = (1/L^3) sum_{k != 0} cos(k.n) / sum_d 4 sin^2(k_d / 2).            */
void orc_greens(int L, double G[4]) {
    double *s = (double *)malloc((size_t)L * sizeof(double));
    double *cs = (double *)malloc((size_t)L * sizeof(double));
    const double pi = 3.14159265358979323846;
    for (int m = 0; m < L; ++m) {
        double h = sin(pi * m / L);
        s[m] = 4.0 * h * h;
        cs[m] = cos(2.0 * pi * m / L);
    }
    for (int t = 0; t < 4; ++t) G[t] = 0.0;
    for (int mz = 0; mz < L; ++mz)
        for (int my = 0; my < L; ++my)
            for (int mx = 0; mx < L; ++mx) {
                if (mx == 0 && my == 0 && mz == 0) continue;
                double inv = 1.0 / (s[mx] + s[my] + s[mz]);
                G[0] += inv;
                G[1] += cs[mx] * inv;
                G[2] += cs[mx] * cs[my] * inv;
                G[3] += cs[mx] * cs[my] * cs[mz] * inv;
            }
    double Ns = (double)L * L * L;
    for (int t = 0; t < 4; ++t) G[t] /= Ns;
    free(s);
    free(cs);
}

/* Self-energy sum of the 8 interpolated corner charges of one unit charge in
 * its cell: S = sum_{o,o'} w_o w_o' G(o - o').  The pair sums factor per axis:
 * equal corners (m_d = 0) give (1-f)^2 + f^2 = 1 - beta, different corners give
 * beta = 2 f (1 - f); G depends on the number of differing axes only. */
void orc_self_sum(const double G[4], const double f[3], double *S, double dS[3]) {
    double beta[3], alpha[3], dbeta[3];
    for (int d = 0; d < 3; ++d) {
        beta[d] = 2.0 * f[d] * (1.0 - f[d]);
        alpha[d] = 1.0 - beta[d];
        dbeta[d] = 2.0 - 4.0 * f[d];
    }
    double s = 0.0, ds[3] = {0.0, 0.0, 0.0};
    for (int m = 0; m < 8; ++m) {
        int mb[3] = {m & 1, (m >> 1) & 1, (m >> 2) & 1};
        double g = G[mb[0] + mb[1] + mb[2]];
        double fac[3], dfac[3];
        for (int d = 0; d < 3; ++d) {
            fac[d] = mb[d] ? beta[d] : alpha[d];
            dfac[d] = mb[d] ? dbeta[d] : -dbeta[d];
        }
        s += g * fac[0] * fac[1] * fac[2];
        ds[0] += g * dfac[0] * fac[1] * fac[2];
        ds[1] += g * fac[0] * dfac[1] * fac[2];
        ds[2] += g * fac[0] * fac[1] * dfac[2];
    }
    *S = s;
    for (int d = 0; d < 3; ++d) dS[d] = ds[d];
}

/* Periodic lattice Green's function at an offset n with every component in
 * {-1, 0, 1}: by cubic symmetry it depends only on how many components are
 * nonzero (G[0..3] = G(000), G(100), G(110), G(111)). */
static double green_near(const double G[4], const long n[3]) {
    int k = 0;
    for (int d = 0; d < 3; ++d) k += n[d] != 0;
    return G[k];
}

/* Direct subtraction of the self influence (section "Self energy
 * interaction", eq. direct-subtraction, whose printed form is garbled; the
 * reading): the ion's own linearly assigned charges q w_m at the 8 corners
 * c + m of its cell produce on each link (u, d) of that cell the displacement
 * field of a homogeneous lattice,
 *   D_self_d(u) = -(q/a^2) sum_m w_m [G(u + e_d - c - m) - G(u - c - m)]
 * (phi = q G/(a eps) of eq. greens, D = -eps grad phi: eps drops out), and its
 * field there is D_self/eps of that link (the permittivity of the link
 * between the two vertices, as the equation has it).  The self force is the
 * force interpolation of that field,
 *   Fself_d = q sum_{4 d-links} w w eta_link D_self_d(link).
 * With the same eps on the 12 edges this is the Green's-function self force. */
static void self_force_direct(int L, double a, double q, const long c[3], const double f[3],
                              const double *eta, const double G[4], double Fself[3]) {
    size_t Ns = (size_t)L * L * L;
    for (int d = 0; d < 3; ++d) {
        int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
        double s = 0.0;
        for (int o2 = 0; o2 < 2; ++o2)
            for (int o1 = 0; o1 < 2; ++o1) {
                long uo[3] = {0, 0, 0};  /* u - c */
                uo[d1] = o1;
                uo[d2] = o2;
                double Dself = 0.0;
                for (int m = 0; m < 8; ++m) {
                    long mb[3] = {m & 1, (m >> 1) & 1, (m >> 2) & 1};
                    double w = wgt((int)mb[0], f[0]) * wgt((int)mb[1], f[1]) * wgt((int)mb[2], f[2]);
                    long nA[3], nB[3];
                    for (int k = 0; k < 3; ++k) {
                        nB[k] = uo[k] - mb[k];
                        nA[k] = nB[k] + (k == d);
                    }
                    Dself += w * (green_near(G, nA) - green_near(G, nB));
                }
                Dself *= -q / (a * a);
                long x[3] = {c[0] + uo[0], c[1] + uo[1], c[2] + uo[2]};
                size_t l = (size_t)d * Ns + site(L, x[0], x[1], x[2]);
                s += wgt(o1, f[d1]) * wgt(o2, f[d2]) * eta[l] * Dself;
            }
        Fself[d] = q * s;
    }
}

/* Forces on the ions (eq. force without the v x B term, which the paper drops;
 * reading: the sign is F = +q E, from eq. maggs:eq:force with dA/dt = -D/eps).
 *  - lattice part: E_d = eta_d D_d on the 4 d-links of the ion's cell, with the
 *    transverse linear weights (the partner of the current assignment);
 *  - self-force: U_self = q^2 S(f) / (2 eps_cell a) with the lattice Green's
 *    function (phi = q G/(a eps), section "Self energy interaction"), and
 *    F_self = -dU_self/dr is subtracted;
 *  - dipole correction (section "Periodicity"): the uniform mode of D equals
 *    -P/V, so the lattice field carries -P/(V eps) on every ion; adding
 *    q P_d/(V eps_h_d) removes it (metallic boundary at infinity).
 * scheme 0: the Green's-function self force; scheme 1: direct subtraction
 * (self_force_direct).  Uself is the Green's-function self energy in both. */
void orc_forces(int L, double a, int n, const double *q, const double *r, const double *D,
                const double *eta, const double *eps_cell, const double eps_h[3],
                const double G[4], const double P[3], int scheme, double *F, double *Uself) {
    size_t Ns = (size_t)L * L * L;
    double V = pow((double)L * a, 3);
    for (int i = 0; i < n; ++i) {
        long kc[3], c[3];
        double f[3];
        for (int d = 0; d < 3; ++d) fold(r[3 * i + d], a, L, &kc[d], &c[d], &f[d]);
        double Flat[3];
        for (int d = 0; d < 3; ++d) {
            int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
            double s = 0.0;
            for (int o2 = 0; o2 < 2; ++o2)
                for (int o1 = 0; o1 < 2; ++o1) {
                    long x[3] = {c[0], c[1], c[2]};
                    x[d1] += o1;
                    x[d2] += o2;
                    size_t l = (size_t)d * Ns + site(L, x[0], x[1], x[2]);
                    s += wgt(o1, f[d1]) * wgt(o2, f[d2]) * eta[l] * D[l];
                }
            Flat[d] = q[i] * s;
        }
        double ec = eps_cell[site(L, c[0], c[1], c[2])];
        double S, dS[3];
        orc_self_sum(G, f, &S, dS);
        double pref = q[i] * q[i] / (2.0 * ec * a);
        if (Uself) Uself[i] = pref * S;
        double Fd[3];
        if (scheme == 1) self_force_direct(L, a, q[i], c, f, eta, G, Fd);
        for (int d = 0; d < 3; ++d) {
            double Fself = scheme == 1 ? Fd[d] : -pref * dS[d] / a;
            F[3 * i + d] = Flat[d] - Fself + q[i] * P[d] / (V * eps_h[d]);
        }
    }
}

/* Field energy 1/2 sum D^2/eps (eq. lagrangian, eq. finalpartitionfunction) plus
 * the magnetic part (c^2/2) sum B^2 in the leapfrog's shadow form
 * B^{n+1/2} . B^{n+3/2}, with B^{n+3/2} formed transiently; U_self is the sum
 * of the ion self energies and U_dip = sum_d P_d^2 / (2 V eps_h_d) is the
 * energy of the uniform mode removed by the dipole correction. */
void orc_energy(int L, double a, double dt, double c, const double *eta, const double *D,
                const double *B, double U_self, const double P[3], const double eps_h[3],
                double out[5]) {
    size_t M = 3 * (size_t)L * L * L;
    double a3 = a * a * a;
    double V = pow((double)L * a, 3);
    double *Bn = (double *)malloc(M * sizeof(double));
    memcpy(Bn, B, M * sizeof(double));
    orc_faraday(L, a, dt, eta, D, Bn);
    double we = 0.0, wb = 0.0;
    for (size_t t = 0; t < M; ++t) {
        we += eta[t] * D[t] * D[t];
        wb += B[t] * Bn[t];
    }
    we *= 0.5 * a3;
    wb *= 0.5 * c * c * a3;
    double ud = 0.0;
    for (int d = 0; d < 3; ++d) ud += P[d] * P[d] / (2.0 * V * eps_h[d]);
    out[0] = we;
    out[1] = wb;
    out[2] = U_self;
    out[3] = ud;
    out[4] = we + wb - U_self - ud;
    free(Bn);
}

/* ------------------------------------------------ counter-based displacements */

/* Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC 2011): each round
 * multiplies words 0 and 2 by fixed odd constants, and the 64-bit products'
 * halves are xored with words 1 and 3 and the round key; the key is bumped by
 * the Weyl constants before every round but the first. */
void orc_philox4x32_10(const unsigned int ctr[4], const unsigned int key[2], unsigned int out[4]) {
    unsigned long long m0 = 0xD2511F53ull, m1 = 0xCD9E8D57ull;
    unsigned int x[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    unsigned int k[2] = {key[0], key[1]};
    for (int rnd = 0; rnd < 10; ++rnd) {
        if (rnd) {
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        unsigned long long a = m0 * (unsigned long long)x[0];
        unsigned long long b = m1 * (unsigned long long)x[2];
        unsigned int y0 = (unsigned int)(b >> 32) ^ x[1] ^ k[0];
        unsigned int y1 = (unsigned int)b;
        unsigned int y2 = (unsigned int)(a >> 32) ^ x[3] ^ k[1];
        unsigned int y3 = (unsigned int)a;
        x[0] = y0;
        x[1] = y1;
        x[2] = y2;
        x[3] = y3;
    }
    for (int t = 0; t < 4; ++t) out[t] = x[t];
}

/* Displacements of n ions at step t from the stream of `seed`: per ion two
 * Philox calls with counters (i, t, 0, 0) and (i, t, 1, 0), key = (low, high
 * 32 bits of seed); each call gives two 53-bit uniforms in [0, 1) from word
 * pairs (w0, w1), (w2, w3) as ((wa >> 5) 2^26 + (wb >> 6)) / 2^53, turned into
 * normals by Box-Muller with radius sqrt(-2 log(1 - ua)) and angle 2 pi ub
 * (cosine, then sine).  The first call gives x and y, the second z. */
void orc_seeded_displacements(unsigned long long seed, int t, int n, double sigma, double *out) {
    const double two_pi = 6.283185307179586476925286766559;
    unsigned int key[2] = {(unsigned int)(seed & 0xffffffffull), (unsigned int)(seed >> 32)};
    for (int i = 0; i < n; ++i) {
        double z[4];
        for (int j = 0; j < 2; ++j) {
            unsigned int ctr[4] = {(unsigned int)i, (unsigned int)t, (unsigned int)j, 0u};
            unsigned int w[4];
            orc_philox4x32_10(ctr, key, w);
            double ua = ((double)(w[0] >> 5) * 67108864.0 + (double)(w[1] >> 6)) / 9007199254740992.0;
            double ub = ((double)(w[2] >> 5) * 67108864.0 + (double)(w[3] >> 6)) / 9007199254740992.0;
            double rad = sqrt(-2.0 * log(1.0 - ua));
            z[2 * j] = rad * cos(two_pi * ub);
            z[2 * j + 1] = rad * sin(two_pi * ub);
        }
        out[3 * i] = sigma * z[0];
        out[3 * i + 1] = sigma * z[1];
        out[3 * i + 2] = sigma * z[2];
    }
}
