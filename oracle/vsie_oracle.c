/*
 * FP64 reference ("oracle") for the discretised nested VSIE operator.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled with gcc into
 * oracle/liboracle.so and is loaded by the tests, by the smoke check and by
 * the CPU-baseline leg of the benchmark.  The GPU library never links or calls
 * it, and it shares no code, header or constant with the GPU library.
 *
 * What is computed (paper, section "Numerical discretization"): collocation at
 * element centroids with P0 basis functions and a one-point (midpoint)
 * quadrature for every integral of the final VSIE (Theorem 3, eq. "eq_vsie").
 * For a collocation point x and a source element j with centroid y_j:
 *
 *   volume source  : -G(x,y_j) * sV_j  +  grad_x G(x,y_j) . gT_j
 *                    sV_j = |cell| (beta - k0^2 alpha)(y_j)     single layer V
 *                    gT_j = |cell| grad alpha(y_j)               adjoint double layer T
 *   surface source :  dG/dn_y(x,y_j) * dK_j                      double layer K
 *                    dK_j = |face| * (alpha jump on the face), n_j the face normal
 *
 * with G = exp(i k0 r)/(4 pi r) (eq. "eq_greens_function"),
 *      grad_x G = F(r) (x - y),   dG/dn_y = grad_y G . n = F(r) (y - x) . n,
 *      F(r) = exp(i k0 r) (i k0 r - 1) / (4 pi r^3)   (derivative of G, divided by r).
 *
 * Every sum over sources is a plain loop with Neumaier-compensated
 * accumulation of the real and imaginary parts.  Complex vectors are
 * interleaved (re, im) doubles, column-major with leading dimension = length.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

typedef double complex cplx;

/* Neumaier (improved Kahan) compensated summation of one real stream. */
typedef struct { double s, c; } nsum;
static inline void nsum_add(nsum *a, double v) {
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}
static inline double nsum_get(const nsum *a) { return a->s + a->c; }

/* G(r) and F(r) for r > 0. */
static inline void green(double k0, double r, cplx *G, cplx *F) {
    const double four_pi = 4.0 * M_PI;
    cplx e = cexp(I * k0 * r);
    *G = e / (four_pi * r);
    *F = e * (I * k0 * r - 1.0) / (four_pi * r * r * r);
}

/* Kernel value kappa(x, j) of one source for one collocation point. */
static inline cplx kappa(double k0, double xt, double yt, double zt,
                         int is_surface, double px, double py, double pz,
                         double sV, double gx, double gy, double gz,
                         double nx, double ny, double nz, double dK) {
    double dx = xt - px, dy = yt - py, dz = zt - pz;
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    cplx G, F;
    green(k0, r, &G, &F);
    if (is_surface) {
        /* dG/dn_y = F(r) (y - x) . n */
        double ymx_n = -(dx * nx + dy * ny + dz * nz);
        return F * ymx_n * dK;
    }
    /* -G sV + grad_x G . gT,  grad_x G = F(r) (x - y) */
    return -G * sV + F * (dx * gx + dy * gy + dz * gz);
}

/*
 * out[i, c] = sum over sources j (j != i when exclude_self) of kappa(t_i, j) * x[j, c]
 *
 * Sources: n_s elements, the first n_vol of them volume cells and the rest
 * surface elements.  sV, gT (3 x n_vol SoA) describe the volume cells; nrm
 * (3 x n_srf SoA) and dK the surface elements.  Targets t are n_t points.
 * rows != NULL restricts the targets to t[rows[i]] (i < n_rows) and writes
 * out[i, c]; exclusion then compares rows[i] with j.
 */
void vo_apply(int64_t n_t, const double *tx, const double *ty, const double *tz,
              const int64_t *rows, int64_t n_rows,
              int64_t n_vol, int64_t n_s, const double *px, const double *py, const double *pz,
              const double *sV, const double *gx, const double *gy, const double *gz,
              const double *nx, const double *ny, const double *nz, const double *dK,
              double k0, int exclude_self, int64_t nrhs,
              const double *x, double *out) {
    int64_t nt = rows ? n_rows : n_t;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t ii = 0; ii < nt; ++ii) {
        int64_t i = rows ? rows[ii] : ii;
        for (int64_t c = 0; c < nrhs; ++c) {
            nsum re = {0, 0}, im = {0, 0};
            const double *xc = x + 2 * c * n_s;
            for (int64_t j = 0; j < n_s; ++j) {
                if (exclude_self && j == i) continue;
                int surf = j >= n_vol;
                int64_t q = surf ? j - n_vol : j;
                cplx kv = surf
                    ? kappa(k0, tx[i], ty[i], tz[i], 1, px[j], py[j], pz[j], 0, 0, 0, 0,
                            nx[q], ny[q], nz[q], dK[q])
                    : kappa(k0, tx[i], ty[i], tz[i], 0, px[j], py[j], pz[j], sV[q], gx[q], gy[q],
                            gz[q], 0, 0, 0, 0);
                cplx xv = xc[2 * j] + I * xc[2 * j + 1];
                cplx p = kv * xv;
                nsum_add(&re, creal(p));
                nsum_add(&im, cimag(p));
            }
            out[2 * (c * nt + ii)] = nsum_get(&re);
            out[2 * (c * nt + ii) + 1] = nsum_get(&im);
        }
    }
}

/*
 * Adjoint sums, straight from the definition of the conjugate transpose:
 * out[j, c] = sum over targets i (i != j when exclude_self) of conj(kappa(t_i, j)) * lam[i, c]
 * for every source j.
 */
void vo_apply_adjoint(int64_t n_t, const double *tx, const double *ty, const double *tz,
                      int64_t n_vol, int64_t n_s, const double *px, const double *py,
                      const double *pz, const double *sV, const double *gx, const double *gy,
                      const double *gz, const double *nx, const double *ny, const double *nz,
                      const double *dK, double k0, int exclude_self, int64_t nrhs,
                      const double *lam, double *out) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < n_s; ++j) {
        int surf = j >= n_vol;
        int64_t q = surf ? j - n_vol : j;
        for (int64_t c = 0; c < nrhs; ++c) {
            nsum re = {0, 0}, im = {0, 0};
            const double *lc = lam + 2 * c * n_t;
            for (int64_t i = 0; i < n_t; ++i) {
                if (exclude_self && i == j) continue;
                cplx kv = surf
                    ? kappa(k0, tx[i], ty[i], tz[i], 1, px[j], py[j], pz[j], 0, 0, 0, 0,
                            nx[q], ny[q], nz[q], dK[q])
                    : kappa(k0, tx[i], ty[i], tz[i], 0, px[j], py[j], pz[j], sV[q], gx[q], gy[q],
                            gz[q], 0, 0, 0, 0);
                cplx p = conj(kv) * (lc[2 * i] + I * lc[2 * i + 1]);
                nsum_add(&re, creal(p));
                nsum_add(&im, cimag(p));
            }
            out[2 * (c * n_s + j)] = nsum_get(&re);
            out[2 * (c * n_s + j) + 1] = nsum_get(&im);
        }
    }
}

/*
 * Source-side reductions used by the adjoint-state gradient:
 *   z[j, c]    = sum_i conj(G(r_ij)) lam[i, c]
 *   Z[j, c, :] = sum_i conj(F(r_ij)) (t_i - y_j) lam[i, c]
 * over targets i (i != j when exclude_self).  Z is stored as 3 consecutive
 * complex blocks of length n_s per right-hand side: Z[(3c + a) n_s + j].
 */
void vo_source_sums(int64_t n_t, const double *tx, const double *ty, const double *tz,
                    int64_t n_s, const double *px, const double *py, const double *pz,
                    double k0, int exclude_self, int64_t nrhs, const double *lam,
                    double *z, double *Z) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < n_s; ++j) {
        for (int64_t c = 0; c < nrhs; ++c) {
            nsum zr = {0, 0}, zi = {0, 0};
            nsum Zr[3] = {{0, 0}, {0, 0}, {0, 0}}, Zi[3] = {{0, 0}, {0, 0}, {0, 0}};
            const double *lc = lam + 2 * c * n_t;
            for (int64_t i = 0; i < n_t; ++i) {
                if (exclude_self && i == j) continue;
                double d[3] = {tx[i] - px[j], ty[i] - py[j], tz[i] - pz[j]};
                double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                cplx G, F;
                green(k0, r, &G, &F);
                cplx l = lc[2 * i] + I * lc[2 * i + 1];
                cplx a = conj(G) * l;
                nsum_add(&zr, creal(a));
                nsum_add(&zi, cimag(a));
                for (int k = 0; k < 3; ++k) {
                    cplx b = conj(F) * d[k] * l;
                    nsum_add(&Zr[k], creal(b));
                    nsum_add(&Zi[k], cimag(b));
                }
            }
            z[2 * (c * n_s + j)] = nsum_get(&zr);
            z[2 * (c * n_s + j) + 1] = nsum_get(&zi);
            for (int k = 0; k < 3; ++k) {
                Z[2 * ((3 * c + k) * n_s + j)] = nsum_get(&Zr[k]);
                Z[2 * ((3 * c + k) * n_s + j) + 1] = nsum_get(&Zi[k]);
            }
        }
    }
}

/*
 * Dense off-diagonal matrix: A[i*n + j] = kappa(p_i, j) for i != j, 0 on the
 * diagonal (the caller adds the diagonal).  Row-major, interleaved complex.
 */
void vo_assemble(int64_t n_vol, int64_t n, const double *px, const double *py, const double *pz,
                 const double *sV, const double *gx, const double *gy, const double *gz,
                 const double *nx, const double *ny, const double *nz, const double *dK,
                 double k0, double *A) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            cplx kv = 0;
            if (j != i) {
                int surf = j >= n_vol;
                int64_t q = surf ? j - n_vol : j;
                kv = surf ? kappa(k0, px[i], py[i], pz[i], 1, px[j], py[j], pz[j], 0, 0, 0, 0,
                                  nx[q], ny[q], nz[q], dK[q])
                          : kappa(k0, px[i], py[i], pz[i], 0, px[j], py[j], pz[j], sV[q], gx[q],
                                  gy[q], gz[q], 0, 0, 0, 0);
            }
            A[2 * (i * n + j)] = creal(kv);
            A[2 * (i * n + j) + 1] = cimag(kv);
        }
    }
}

/* Number of OpenMP threads the oracle runs with (0 when built without OpenMP). */
int vo_num_threads(void) {
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 0;
#endif
}
