/*
 * spgm_oracle.c -- plain, slow, double-precision CPU reference ("the oracle") for the
 * stochastic proximal-gradient (SPGM) near-field MIMO projector of
 * O. Oral, "Fast Regularized 3D Near-Field MIMO Imaging Using Stochastic Proximal
 * Gradient Method" (arXiv 2509.00774).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call this
 * file: it is used by the test-suite, by the package's smoke check and by the benchmark's
 * CPU-baseline leg.  It shares no code, header, table or helper with the HIP path.
 *
 * Every routine is written from the paper's definitions, in its notation, with no
 * blocking, fusion or reordering beyond what the definition states:
 *   - observation model y = A s + w                                   (Sec. II, Eq. 1)
 *   - entry A_{m,n} = p(f_m) exp(-j 2 pi f_m (|r_Tm - r_n| + |r_Rm - r_n|) / c)
 *                     / (4 pi |r_Tm - r_n| |r_Rm - r_n|),
 *     with transmitters and receivers given by their 3-D positions      (Sec. II, Eq. 2)
 *   - data fidelity D(s) = (1/2M) |y - A s|^2 = mean_m D_m(s),
 *     D_m(s) = 1/2 |y_m - sum_n A_{m,n} s_n|^2                         (Sec. III, Eq. 4)
 *   - PGM iteration s <- prox_{alpha R}(s - eta grad D(s)), alpha = lambda eta   (Sec. IV, Eq. 5)
 *   - SPGM gradient = gradient of (1/B) sum_{m<B} D_{b_m}(s)          (Sec. IV-A, Eq. 6)
 *   - other regularisers in place of l1 (extension noted in Sec. III): elastic net and total
 *     variation of the magnitudes, with their readings in the section that defines them
 *
 * Readings where the paper is silent (each one is listed in the design notes):
 *   - row index m = (i_f * T + i_t) * R + i_r  (frequency-major, then Tx, then Rx);
 *   - voxel index n = (i_z * ny + i_y) * nx + i_x, voxel centre
 *     r = centre + (i - (n_dim - 1)/2) * pitch per axis;
 *   - complex numbers are interleaved (re, im) doubles;
 *   - the gradient of D_m with respect to the complex unknown is the Wirtinger gradient
 *     conj(A_m)^T (A_m s - y_m), so the minibatch gradient is (1/B) A_B^H (A_B s - y_B);
 *   - R(s) = sum_n |s_n| (complex modulus), whose prox is the complex soft threshold
 *     S_a(v) = v * max(0, 1 - a/|v|), with S_a(v) = 0 whenever |v| <= a.
 *
 * Build: gcc -O2 -fopenmp -fPIC -shared (no fast-math), see oracle/build.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double PI = 3.14159265358979323846264338327950288;

typedef struct {
    int32_t n_tx, n_rx, n_freq;   /* T, R, F */
    int32_t nx, ny, nz;           /* voxel grid */
    const double *tx_xyz;         /* T x 3, metres */
    const double *rx_xyz;         /* R x 3, metres */
    const double *freq_hz;        /* F */
    const double *pulse;          /* F x 2 (re, im) = p(f); NULL means p = 1 */
    double centre[3];             /* grid centre, metres */
    double pitch[3];              /* voxel pitch, metres */
    double c;                     /* propagation speed, m/s */
} ora_geometry;

int ora_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int64_t ora_num_rows(const ora_geometry *g) {
    return (int64_t)g->n_freq * g->n_tx * g->n_rx;
}

int64_t ora_num_voxels(const ora_geometry *g) {
    return (int64_t)g->nx * g->ny * g->nz;
}

/* Voxel centre r_n on the regular grid (Sec. II: r_n = [x_n, y_n, z_n]). */
void ora_voxel_position(const ora_geometry *g, int64_t n, double r[3]) {
    int64_t ix = n % g->nx;
    int64_t iy = (n / g->nx) % g->ny;
    int64_t iz = n / ((int64_t)g->nx * g->ny);
    r[0] = g->centre[0] + ((double)ix - 0.5 * (g->nx - 1)) * g->pitch[0];
    r[1] = g->centre[1] + ((double)iy - 0.5 * (g->ny - 1)) * g->pitch[1];
    r[2] = g->centre[2] + ((double)iz - 0.5 * (g->nz - 1)) * g->pitch[2];
}

/* Split measurement index m into (frequency, transmitter, receiver). */
static void decode_row(const ora_geometry *g, int64_t m, int64_t *i_f, int64_t *i_t, int64_t *i_r) {
    *i_r = m % g->n_rx;
    *i_t = (m / g->n_rx) % g->n_tx;
    *i_f = m / ((int64_t)g->n_rx * g->n_tx);
}

static double dist3(const double *a, const double *b) {
    double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return sqrt(dx * dx + dy * dy + dz * dz);
}

/* Entry A_{m,n} of the observation matrix, Eq. 2, written out term by term. */
void ora_entry(const ora_geometry *g, int64_t m, int64_t n, double out[2]) {
    int64_t i_f, i_t, i_r;
    double rn[3];
    decode_row(g, m, &i_f, &i_t, &i_r);
    ora_voxel_position(g, n, rn);
    const double f = g->freq_hz[i_f];
    const double d_t = dist3(g->tx_xyz + 3 * i_t, rn);   /* |r_Tm - r_n| */
    const double d_r = dist3(g->rx_xyz + 3 * i_r, rn);   /* |r_Rm - r_n| */
    const double arg = -2.0 * PI * f * (d_t + d_r) / g->c;
    const double amp = 1.0 / (4.0 * PI * d_t * d_r);
    const double e_re = cos(arg) * amp;
    const double e_im = sin(arg) * amp;
    const double p_re = g->pulse ? g->pulse[2 * i_f] : 1.0;
    const double p_im = g->pulse ? g->pulse[2 * i_f + 1] : 0.0;
    out[0] = p_re * e_re - p_im * e_im;
    out[1] = p_re * e_im + p_im * e_re;
}

/* Dense rows of A: A_out[j][n] = A_{rows[j], n}, B x N complex. Tiny grids only. */
void ora_dense(const ora_geometry *g, const int32_t *rows, int32_t B, double *A_out) {
    const int64_t N = ora_num_voxels(g);
#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < B; ++j)
        for (int64_t n = 0; n < N; ++n)
            ora_entry(g, rows[j], n, A_out + 2 * ((int64_t)j * N + n));
}

/* y_j = sum_n A_{rows[j], n} s_n   (Eq. 1 restricted to the minibatch rows). */
void ora_forward(const ora_geometry *g, const int32_t *rows, int32_t B, const double *s, double *y) {
    const int64_t N = ora_num_voxels(g);
#pragma omp parallel for schedule(dynamic, 4)
    for (int32_t j = 0; j < B; ++j) {
        double acc_re = 0.0, acc_im = 0.0, a[2];
        for (int64_t n = 0; n < N; ++n) {
            ora_entry(g, rows[j], n, a);
            acc_re += a[0] * s[2 * n] - a[1] * s[2 * n + 1];
            acc_im += a[0] * s[2 * n + 1] + a[1] * s[2 * n];
        }
        y[2 * j] = acc_re;
        y[2 * j + 1] = acc_im;
    }
}

/* Same sum over an explicit list of (voxel index, value) pairs; terms with s_n = 0
 * contribute nothing, so for a sparse scene this equals ora_forward exactly up to
 * summation order.  Used to synthesise measurements of sparse scenes. */
void ora_forward_sparse(const ora_geometry *g, const int32_t *rows, int32_t B,
                        const int64_t *idx, const double *vals, int64_t nnz, double *y) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int32_t j = 0; j < B; ++j) {
        double acc_re = 0.0, acc_im = 0.0, a[2];
        for (int64_t k = 0; k < nnz; ++k) {
            ora_entry(g, rows[j], idx[k], a);
            acc_re += a[0] * vals[2 * k] - a[1] * vals[2 * k + 1];
            acc_im += a[0] * vals[2 * k + 1] + a[1] * vals[2 * k];
        }
        y[2 * j] = acc_re;
        y[2 * j + 1] = acc_im;
    }
}

/* out_n = sum_j conj(A_{rows[j], n}) r_j  (the conjugate-transpose product A_B^H r). */
void ora_adjoint(const ora_geometry *g, const int32_t *rows, int32_t B, const double *r, double *out) {
    const int64_t N = ora_num_voxels(g);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t n = 0; n < N; ++n) {
        double acc_re = 0.0, acc_im = 0.0, a[2];
        for (int32_t j = 0; j < B; ++j) {
            ora_entry(g, rows[j], n, a);
            /* conj(a) * r = (a_re - i a_im)(r_re + i r_im) */
            acc_re += a[0] * r[2 * j] + a[1] * r[2 * j + 1];
            acc_im += a[0] * r[2 * j + 1] - a[1] * r[2 * j];
        }
        out[2 * n] = acc_re;
        out[2 * n + 1] = acc_im;
    }
}

/* The same sum for a listed subset of voxels: out_k = sum_j conj(A_{rows[j], idx[k]}) r_j. */
void ora_adjoint_voxels(const ora_geometry *g, const int32_t *rows, int32_t B, const double *r,
                        const int64_t *idx, int64_t nidx, double *out) {
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = 0; k < nidx; ++k) {
        double acc_re = 0.0, acc_im = 0.0, a[2];
        for (int32_t j = 0; j < B; ++j) {
            ora_entry(g, rows[j], idx[k], a);
            acc_re += a[0] * r[2 * j] + a[1] * r[2 * j + 1];
            acc_im += a[0] * r[2 * j + 1] - a[1] * r[2 * j];
        }
        out[2 * k] = acc_re;
        out[2 * k + 1] = acc_im;
    }
}

/* Proximal operator of a * sum_n |s_n| (complex soft threshold), in place. */
void ora_prox_l1(double *v, int64_t N, double a) {
    for (int64_t n = 0; n < N; ++n) {
        const double mag = hypot(v[2 * n], v[2 * n + 1]);
        if (mag <= a) {
            v[2 * n] = 0.0;
            v[2 * n + 1] = 0.0;
        } else {
            const double scale = 1.0 - a / mag;
            v[2 * n] *= scale;
            v[2 * n + 1] *= scale;
        }
    }
}

/* Minibatch gradient of (1/B) sum_j D_{rows[j]}(s) (Eq. 6): (1/B) A_B^H (A_B s - y_B).
 * y is the full measurement vector (length M), gathered by rows. */
void ora_stochastic_gradient(const ora_geometry *g, const int32_t *rows, int32_t B,
                             const double *y, const double *s, double *grad) {
    const int64_t N = ora_num_voxels(g);
    double *res = (double *)malloc(sizeof(double) * 2 * (size_t)B);
    ora_forward(g, rows, B, s, res);
    for (int32_t j = 0; j < B; ++j) {
        res[2 * j] -= y[2 * (int64_t)rows[j]];
        res[2 * j + 1] -= y[2 * (int64_t)rows[j] + 1];
    }
    ora_adjoint(g, rows, B, res, grad);
    for (int64_t n = 0; n < 2 * N; ++n) grad[n] /= (double)B;
    free(res);
}

/* One SPGM iteration (Eq. 5 with the gradient of Eq. 6):
 * s <- prox_{alpha |.|_1}(s - eta * grad), in place. */
void ora_step(const ora_geometry *g, const int32_t *rows, int32_t B, const double *y,
              double *s, double eta, double alpha) {
    const int64_t N = ora_num_voxels(g);
    double *grad = (double *)malloc(sizeof(double) * 2 * (size_t)N);
    ora_stochastic_gradient(g, rows, B, y, s, grad);
    for (int64_t n = 0; n < 2 * N; ++n) s[n] -= eta * grad[n];
    ora_prox_l1(s, N, alpha);
    free(grad);
}

/* K SPGM iterations; iteration k uses rows[k*B .. k*B+B-1]. */
void ora_solve(const ora_geometry *g, const int32_t *rows, int32_t K, int32_t B, const double *y,
               double *s, double eta, double alpha) {
    for (int32_t k = 0; k < K; ++k) ora_step(g, rows + (int64_t)k * B, B, y, s, eta, alpha);
}

/* Iterations of Eq. 5 until the termination rule of Sec. V, "the change in the reflectivity
 * magnitudes drops below tol", read as the relative 2-norm change of the magnitude vector:
 * stop after the first iteration k with
 *     || |s^k| - |s^{k-1}| ||_2 < tol || |s^{k-1}| ||_2,
 * compared as sum(diff^2) < tol^2 sum(|s^{k-1}|^2), so the rule is never met while s^{k-1} = 0.
 * At most K iterations (iteration k uses rows[(k-1)*B ...]); tol <= 0 runs all K.  s holds the
 * iterate at the stop; returns the number of iterations performed. */
int32_t ora_solve_tol(const ora_geometry *g, const int32_t *rows, int32_t K, int32_t B, const double *y,
                      double *s, double eta, double alpha, double tol) {
    const int64_t N = ora_num_voxels(g);
    double *prev = (double *)malloc(sizeof(double) * 2 * (size_t)N);
    int32_t done = K;
    for (int32_t k = 0; k < K; ++k) {
        memcpy(prev, s, sizeof(double) * 2 * (size_t)N);
        ora_step(g, rows + (int64_t)k * B, B, y, s, eta, alpha);
        if (tol <= 0.0) continue;
        double diff2 = 0.0, old2 = 0.0;
        for (int64_t n = 0; n < N; ++n) {
            const double m_new = hypot(s[2 * n], s[2 * n + 1]);
            const double m_old = hypot(prev[2 * n], prev[2 * n + 1]);
            diff2 += (m_new - m_old) * (m_new - m_old);
            old2 += m_old * m_old;
        }
        if (diff2 < tol * tol * old2) {
            done = k + 1;
            break;
        }
    }
    free(prev);
    return done;
}

/* ------------------------------------------------------------------------------------------
 * Other regularisers (the paper notes the method extends to other regularisation functionals,
 * Sec. III); the prox replaces the complex soft threshold in the iteration of Eq. 5.
 * Readings (no formula in the paper; listed in the design notes):
 *   - elastic net R(s) = sum_n |s_n| + (mu/2) sum_n |s_n|^2, whose prox is the soft threshold
 *     followed by the scaling 1/(1 + a mu);
 *   - total variation of the magnitudes, R(s) = TV(|s|) with the isotropic 3-D TV
 *     TV(u) = sum_n || (D u)_n ||_2, (D u)_{n,d} = u_{n+e_d} - u_n inside the grid and 0 on the
 *     upper face of axis d; the prox keeps the phase and replaces the magnitude by the
 *     non-negative solution of  min_u 1/2 ||u - |v| ||^2 + a TV(u),  computed with the fast
 *     gradient projection on the dual (Beck & Teboulle 2009) for a given number of iterations:
 *         u = P+(b - a D^T w),  w <- P_ball(r + D u / (12 a)),  r <- w + ((t_k - 1)/t_{k+1})(w - w_prev),
 *     t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2, t_1 = 1, step 1/(12 a) from ||D||^2 <= 12 in 3-D.
 * ------------------------------------------------------------------------------------------ */

/* Forward-difference gradient: w[d*N + n] = u[n + e_d] - u[n] inside, 0 on the upper face. */
void ora_grad3(int32_t nx, int32_t ny, int32_t nz, const double *u, double *w) {
    const int64_t N = (int64_t)nx * ny * nz;
    for (int32_t iz = 0; iz < nz; ++iz)
        for (int32_t iy = 0; iy < ny; ++iy)
            for (int32_t ix = 0; ix < nx; ++ix) {
                const int64_t n = ((int64_t)iz * ny + iy) * nx + ix;
                w[0 * N + n] = ix + 1 < nx ? u[n + 1] - u[n] : 0.0;
                w[1 * N + n] = iy + 1 < ny ? u[n + nx] - u[n] : 0.0;
                w[2 * N + n] = iz + 1 < nz ? u[n + (int64_t)nx * ny] - u[n] : 0.0;
            }
}

/* Adjoint of ora_grad3: out[n] = sum_d (w_d[n - e_d] if n - e_d is inside) - (w_d[n] if n + e_d is inside). */
void ora_grad3_adjoint(int32_t nx, int32_t ny, int32_t nz, const double *w, double *out) {
    const int64_t N = (int64_t)nx * ny * nz, sy = nx, sz = (int64_t)nx * ny;
    for (int32_t iz = 0; iz < nz; ++iz)
        for (int32_t iy = 0; iy < ny; ++iy)
            for (int32_t ix = 0; ix < nx; ++ix) {
                const int64_t n = ((int64_t)iz * ny + iy) * nx + ix;
                double acc = 0.0;
                if (ix > 0) acc += w[0 * N + n - 1];
                if (ix + 1 < nx) acc -= w[0 * N + n];
                if (iy > 0) acc += w[1 * N + n - sy];
                if (iy + 1 < ny) acc -= w[1 * N + n];
                if (iz > 0) acc += w[2 * N + n - sz];
                if (iz + 1 < nz) acc -= w[2 * N + n];
                out[n] = acc;
            }
}

/* Elastic-net prox in place: v <- S_a(v) / (1 + a mu). */
void ora_prox_elastic(double *v, int64_t N, double a, double mu) {
    ora_prox_l1(v, N, a);
    const double scale = 1.0 / (1.0 + a * mu);
    for (int64_t n = 0; n < 2 * N; ++n) v[n] *= scale;
}

/* Magnitude-TV prox in place on complex v (grid nx x ny x nz), `iters` dual iterations.
 * w_out (3N doubles, may be NULL) receives the final dual field w, from which the returned
 * magnitude is u = max(0, |v| - a D^T w). */
void ora_prox_tv_magnitude(double *v, int32_t nx, int32_t ny, int32_t nz, double a, int32_t iters,
                           double *w_out) {
    const int64_t N = (int64_t)nx * ny * nz;
    double *b = (double *)malloc(sizeof(double) * N);
    double *u = (double *)malloc(sizeof(double) * N);
    double *t = (double *)malloc(sizeof(double) * N);
    double *w = (double *)calloc(3 * (size_t)N, sizeof(double));
    double *w_prev = (double *)calloc(3 * (size_t)N, sizeof(double));
    double *r = (double *)calloc(3 * (size_t)N, sizeof(double));
    double *g = (double *)malloc(sizeof(double) * 3 * N);
    for (int64_t n = 0; n < N; ++n) b[n] = hypot(v[2 * n], v[2 * n + 1]);
    if (a > 0.0) {
        double tk = 1.0;
        for (int32_t k = 0; k < iters; ++k) {
            /* primal point of the extrapolated dual, projected on u >= 0 */
            ora_grad3_adjoint(nx, ny, nz, r, t);
            for (int64_t n = 0; n < N; ++n) u[n] = fmax(0.0, b[n] - a * t[n]);
            /* dual ascent step and projection of every voxel's 3-vector on the unit ball */
            ora_grad3(nx, ny, nz, u, g);
            memcpy(w_prev, w, sizeof(double) * 3 * N);
            for (int64_t n = 0; n < N; ++n) {
                double p0 = r[n] + g[n] / (12.0 * a);
                double p1 = r[N + n] + g[N + n] / (12.0 * a);
                double p2 = r[2 * N + n] + g[2 * N + n] / (12.0 * a);
                const double norm = sqrt(p0 * p0 + p1 * p1 + p2 * p2);
                if (norm > 1.0) {
                    p0 /= norm;
                    p1 /= norm;
                    p2 /= norm;
                }
                w[n] = p0;
                w[N + n] = p1;
                w[2 * N + n] = p2;
            }
            /* momentum */
            const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * tk * tk));
            const double beta = (tk - 1.0) / tn;
            for (int64_t i = 0; i < 3 * N; ++i) r[i] = w[i] + beta * (w[i] - w_prev[i]);
            tk = tn;
        }
        ora_grad3_adjoint(nx, ny, nz, w, t);
        for (int64_t n = 0; n < N; ++n) u[n] = fmax(0.0, b[n] - a * t[n]);
    } else {
        memcpy(u, b, sizeof(double) * N);
    }
    if (w_out) memcpy(w_out, w, sizeof(double) * 3 * N);
    /* keep the phase: v <- u v/|v| (0 where v = 0) */
    for (int64_t n = 0; n < N; ++n) {
        if (b[n] > 0.0) {
            const double scale = u[n] / b[n];
            v[2 * n] *= scale;
            v[2 * n + 1] *= scale;
        } else {
            v[2 * n] = 0.0;
            v[2 * n + 1] = 0.0;
        }
    }
    free(b);
    free(u);
    free(t);
    free(w);
    free(w_prev);
    free(r);
    free(g);
}

/* One iteration of Eq. 5 with the minibatch gradient of Eq. 6 and the prox of the chosen
 * regulariser: kind 0 = l1, 1 = elastic net (mu), 2 = magnitude TV (tv_iters). */
void ora_step_reg(const ora_geometry *g, const int32_t *rows, int32_t B, const double *y, double *s, double eta,
                  double alpha, int32_t kind, double mu, int32_t tv_iters) {
    const int64_t N = ora_num_voxels(g);
    double *grad = (double *)malloc(sizeof(double) * 2 * (size_t)N);
    ora_stochastic_gradient(g, rows, B, y, s, grad);
    for (int64_t n = 0; n < 2 * N; ++n) s[n] -= eta * grad[n];
    if (kind == 1) ora_prox_elastic(s, N, alpha, mu);
    else if (kind == 2) ora_prox_tv_magnitude(s, g->nx, g->ny, g->nz, alpha, tv_iters, NULL);
    else ora_prox_l1(s, N, alpha);
    free(grad);
}
