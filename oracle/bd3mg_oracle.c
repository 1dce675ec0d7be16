/*
 * BD3MG oracle: a plain, slow, FP64 CPU implementation of what the block
 * distributed 3MG method computes for 3D deblurring under depth-variant blur
 * (Chalvidal & Chouzenoux, "Block distributed 3MG algorithm and its
 * application to 3D image restoration", arXiv 2002.02328).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the HIP implementation.
 *
 * Conventions (readings of the paper where it is silent; each is listed with
 * its reason in the design notes of the repository):
 *   - Volumes are [nz][ny][nx], x fastest.  Index (k, j, i).
 *   - H is output-slice indexed (Sec. 3.1: each depth has its own blur
 *     kernel): (Hx)_{k,j,i} = sum_{c,b,a} P_k[c][b][a] x_{k-c, j-b, i-a},
 *     zero padding, same size.  P_k is either separable, P_k[c][b][a] =
 *     gz_k[c] gy_k[b] gx_k[a] with tables stored as g[k][a + r], a in
 *     [-r, r], or a general kernel (the rotated Gaussians of random
 *     variance and rotation that the paper draws per depth) stored as
 *     pk[k][c + rz][b + ry][a + rx].
 *   - V^X, V^Y, V^Z are forward differences whose last difference is 0.
 *   - f is the criterion of Sec. 3.1 (eq. "eq_crit"):
 *       f(x) = 1/2 ||Hx - y||^2 + eta d^2(x, [xmin,xmax]^N)
 *            + lambda sum_n sqrt((V^X x)_n^2 + (V^Y x)_n^2 + delta^2)
 *            + kappa ||V^Z x||^2.
 *   - The block majorant matrix (Sec. 2.2, eq. "maj"; built "following" the
 *     3MG paper as Sec. 3.1 says) is the half-quadratic one:
 *       A(x) = H^T H + 2 eta I + lambda D^T Diag(omega(x)) D + 2 kappa VZ^T VZ,
 *     omega = 1/sqrt((V^X x)^2 + (V^Y x)^2 + delta^2), D = [V^X; V^Y].
 *     A_(S) is its principal submatrix on the block S.
 *   - Worker step (Sec. 2.3, box "Worker", eq. "minimizer"):
 *       D_S = [-grad_S f | d_S],  u = -(D^T A_S D)^+ D^T grad_S f,  d' = D_S u.
 *     d_S is the block's own previous step (0 on its first visit).
 *   - The Moore-Penrose inverse of the 2x2 PSD matrix follows the rank rule of
 *     orc_pinv2 below.
 *
 * Sums are accumulated per slice in plain index order and the per-slice
 * partials are added in slice order, so results do not depend on the number
 * of OpenMP threads.  Compile without floating-point contraction.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int nx, ny, nz;
    int kx, ky, kz;              /* odd kernel sizes */
    const double *gx, *gy, *gz;  /* [nz][kx], [nz][ky], [nz][kz] */
    const double *y;             /* observation, [nz][ny][nx] */
    double lambda, delta, eta, kappa, xmin, xmax;
    int dense;                   /* 1: triple-sum definition of H; 0: separable twin */
    double mu;                   /* curvature inflation of every block majorant (Assumption C); 0: none */
    const double *pk;            /* general kernels [nz][kz][ky][kx] (triple sum), or NULL */
    /* Block step of the ablation study (Sec. 3.2, "Ablation study and
     * comparative analysis"): 0 BD3MG; 1 Async-GD (subspace {-grad}, metric
     * L Id); 2 Async-CG (subspace {-grad, d_prev}, metric L Id); 3 Async-MM
     * (d' = -A_S(x)^{-1} grad_S f by linear BiCG).  mu adds to every metric. */
    int method;
    double lip;                  /* L of the metric L Id (methods 1 and 2) */
    int n_inner;                 /* Async-MM: BiCG iterations at most */
    double tol_inner;            /* Async-MM: stop when ||r_k|| <= tol_inner ||r_0|| (0: never) */
    /* 1: three-dimensional total variation, V^Z inside the root with V^X and
     * V^Y (the generic ||(D x)_n|| form of the TV term); 0: V^X, V^Y only, as
     * in the criterion of Sec. 3.1 */
    int tv3d;
} orc_problem;

#define VOX(p, k, j, i) (((size_t)(k) * (size_t)(p)->ny + (size_t)(j)) * (size_t)(p)->nx + (size_t)(i))

static size_t nvox(const orc_problem *p) { return (size_t)p->nx * p->ny * p->nz; }
static size_t nslice(const orc_problem *p) { return (size_t)p->nx * p->ny; }

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads used by later calls (timing the oracle on one core or on all). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Reusable zero-filled scratch volumes.  A buffer handed out by scratch_get
 * is all zeros; its user zeroes the slices it wrote before scratch_put, so the
 * oracle does not clear whole volumes on every block update.  (Storage only:
 * no arithmetic depends on it.) */
enum { SCR_R, SCR_HU, SCR_HV, SCR_G, SCR_D1, SCR_D2, SCR_DN, SCR_COUNT };
static double *scr_buf[SCR_COUNT];
static size_t scr_cap[SCR_COUNT];

static double *scratch_get(int slot, size_t n)
{
    if (scr_cap[slot] < n) {
        free(scr_buf[slot]);
        scr_buf[slot] = (double *)calloc(n, sizeof(double));
        scr_cap[slot] = n;
    }
    return scr_buf[slot];
}

/* Zero slices [k0, k1) (of S voxels each) of a scratch buffer. */
static void scratch_clear(double *b, int k0, int k1, size_t S)
{
    if (k1 > k0) memset(b + (size_t)k0 * S, 0, (size_t)(k1 - k0) * S * sizeof(double));
}

/* ------------------------------------------------------------------------ */
/* PSF tables.  Sec. 3.1: a depth-variant Gaussian blur.  Each 1-D factor is
 * exp(-a^2 / (2 sigma_k^2)) on a in [-r, r], normalised to sum 1 (so each
 * per-slice 3-D kernel sums to 1).                                           */
void orc_gauss_table(int nz, int k, const double *sigma, double *out)
{
    int r = k / 2;
    for (int z = 0; z < nz; ++z) {
        double s = 0.0;
        for (int a = -r; a <= r; ++a) {
            double v = exp(-(double)(a * a) / (2.0 * sigma[z] * sigma[z]));
            out[(size_t)z * k + (a + r)] = v;
            s += v;
        }
        for (int a = 0; a < k; ++a) out[(size_t)z * k + a] /= s;
    }
}

/* General per-depth kernels of the paper's experiments (Sec. 3.1: each depth
 * has a Gaussian blur of its own variance and rotation): for slice k, an
 * anisotropic Gaussian with in-slice widths sx[k] along the axis rotated by
 * theta[k] from x and sy[k] across it, and width sz[k] along z,
 *   P_k[c][b][a] = exp(-u^2 / (2 sx^2) - v^2 / (2 sy^2) - c^2 / (2 sz^2)) / Z_k,
 *   u = a cos(theta) + b sin(theta),  v = -a sin(theta) + b cos(theta),
 * normalised so that every P_k sums to 1.  out is [nz][kz][kxy][kxy].      */
void orc_rotated_gauss(int nz, int kxy, int kz, const double *sx, const double *sy,
                       const double *theta, const double *sz, double *out)
{
    int r = kxy / 2, rz = kz / 2;
    size_t per = (size_t)kz * kxy * kxy;
    for (int k = 0; k < nz; ++k) {
        double *o = out + (size_t)k * per;
        double ct = cos(theta[k]), st = sin(theta[k]), tot = 0.0;
        for (int c = -rz; c <= rz; ++c)
            for (int b = -r; b <= r; ++b)
                for (int a = -r; a <= r; ++a) {
                    double u = a * ct + b * st, v = -a * st + b * ct;
                    double e = u * u / (2.0 * sx[k] * sx[k]) + v * v / (2.0 * sy[k] * sy[k]) +
                               (double)(c * c) / (2.0 * sz[k] * sz[k]);
                    double w = exp(-e);
                    o[((size_t)(c + rz) * kxy + (b + r)) * kxy + (a + r)] = w;
                    tot += w;
                }
        for (size_t q = 0; q < per; ++q) o[q] /= tot;
    }
}

/* ------------------------------------------------------------------------ */
/* H and its adjoint, restricted to output slices [k0, k1).                  */

/* Kernel weight P_k[c][b][a] (c, b, a centred). */
static double psf_w(const orc_problem *p, int k, int c, int b, int a)
{
    int rx = p->kx / 2, ry = p->ky / 2, rz = p->kz / 2;
    if (p->pk)
        return p->pk[(((size_t)k * p->kz + (c + rz)) * p->ky + (b + ry)) * p->kx + (a + rx)];
    return p->gz[(size_t)k * p->kz + c + rz] * p->gy[(size_t)k * p->ky + b + ry] *
           p->gx[(size_t)k * p->kx + a + rx];
}

/* Triple-sum definition. */
static void H_dense(const orc_problem *p, const double *x, double *out, int k0, int k1)
{
    int rx = p->kx / 2, ry = p->ky / 2, rz = p->kz / 2;
#pragma omp parallel for schedule(static)
    for (int k = k0; k < k1; ++k) {
        for (int j = 0; j < p->ny; ++j)
            for (int i = 0; i < p->nx; ++i) {
                double s = 0.0;
                for (int c = -rz; c <= rz; ++c) {
                    int kk = k - c;
                    if (kk < 0 || kk >= p->nz) continue;
                    for (int b = -ry; b <= ry; ++b) {
                        int jj = j - b;
                        if (jj < 0 || jj >= p->ny) continue;
                        for (int a = -rx; a <= rx; ++a) {
                            int ii = i - a;
                            if (ii < 0 || ii >= p->nx) continue;
                            double w = psf_w(p, k, c, b, a);
                            s += w * x[VOX(p, kk, jj, ii)];
                        }
                    }
                }
                out[VOX(p, k, j, i)] = s;
            }
    }
}

/* (H^T r)_{k,j,i} = sum_{c,b,a} P_{k+c}[c][b][a] r_{k+c, j+b, i+a}. */
static void HT_dense(const orc_problem *p, const double *r, double *out, int k0, int k1)
{
    int rx = p->kx / 2, ry = p->ky / 2, rz = p->kz / 2;
#pragma omp parallel for schedule(static)
    for (int k = k0; k < k1; ++k) {
        for (int j = 0; j < p->ny; ++j)
            for (int i = 0; i < p->nx; ++i) {
                double s = 0.0;
                for (int c = -rz; c <= rz; ++c) {
                    int kk = k + c;
                    if (kk < 0 || kk >= p->nz) continue;
                    for (int b = -ry; b <= ry; ++b) {
                        int jj = j + b;
                        if (jj < 0 || jj >= p->ny) continue;
                        for (int a = -rx; a <= rx; ++a) {
                            int ii = i + a;
                            if (ii < 0 || ii >= p->nx) continue;
                            double w = psf_w(p, kk, c, b, a);
                            s += w * r[VOX(p, kk, jj, ii)];
                        }
                    }
                }
                out[VOX(p, k, j, i)] = s;
            }
    }
}

/* In-slice blur of one slice with the factors of slice m:
 * forward (transpose = 0): out_{j,i} = sum_b gy[b] sum_a gx[a] s_{j-b, i-a}
 * adjoint (transpose = 1): out_{j,i} = sum_b gy[b] sum_a gx[a] s_{j+b, i+a}  */
static void blur_slice(const orc_problem *p, int m, int transpose,
                       const double *s, double *out, double *tmp)
{
    int rx = p->kx / 2, ry = p->ky / 2, nx = p->nx, ny = p->ny;
    int sg = transpose ? 1 : -1;
    const double *gy = p->gy + (size_t)m * p->ky;
    const double *gx = p->gx + (size_t)m * p->kx;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double acc = 0.0;
            for (int a = -rx; a <= rx; ++a) {
                int ii = i + sg * a;
                if (ii < 0 || ii >= nx) continue;
                acc += gx[a + rx] * s[(size_t)j * nx + ii];
            }
            tmp[(size_t)j * nx + i] = acc;
        }
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double acc = 0.0;
            for (int b = -ry; b <= ry; ++b) {
                int jj = j + sg * b;
                if (jj < 0 || jj >= ny) continue;
                acc += gy[b + ry] * tmp[(size_t)jj * nx + i];
            }
            out[(size_t)j * nx + i] = acc;
        }
}

/* Separable twin of H: combine along z with the output slice's gz, then blur
 * in-slice with the output slice's xy factors.  Equal to H_dense up to
 * rounding (the kernel is a product of 1-D factors).                        */
static void H_sep(const orc_problem *p, const double *x, double *out, int k0, int k1)
{
    int rz = p->kz / 2;
    size_t S = nslice(p);
#pragma omp parallel
    {
        double *t = (double *)malloc(S * sizeof(double));
        double *tmp = (double *)malloc(S * sizeof(double));
#pragma omp for schedule(static)
        for (int k = k0; k < k1; ++k) {
            const double *gz = p->gz + (size_t)k * p->kz;
            for (size_t q = 0; q < S; ++q) {
                double acc = 0.0;
                for (int c = -rz; c <= rz; ++c) {
                    int kk = k - c;
                    if (kk < 0 || kk >= p->nz) continue;
                    acc += gz[c + rz] * x[(size_t)kk * S + q];
                }
                t[q] = acc;
            }
            blur_slice(p, k, 0, t, out + (size_t)k * S, tmp);
        }
        free(t);
        free(tmp);
    }
}

/* Separable twin of H^T: blur each input slice m with its own factors
 * (adjoint form), then gather along z with gz_m.                            */
static void HT_sep(const orc_problem *p, const double *r, double *out, int k0, int k1)
{
    int rz = p->kz / 2;
    size_t S = nslice(p);
    int m0 = k0 - rz < 0 ? 0 : k0 - rz;
    int m1 = k1 + rz > p->nz ? p->nz : k1 + rz;
    int nm = m1 - m0;
    if (nm <= 0) return;
    double *bl = (double *)malloc((size_t)nm * S * sizeof(double));
#pragma omp parallel
    {
        double *tmp = (double *)malloc(S * sizeof(double));
#pragma omp for schedule(static)
        for (int m = m0; m < m1; ++m)
            blur_slice(p, m, 1, r + (size_t)m * S, bl + (size_t)(m - m0) * S, tmp);
        free(tmp);
    }
#pragma omp parallel for schedule(static)
    for (int k = k0; k < k1; ++k) {
        for (size_t q = 0; q < S; ++q) {
            double acc = 0.0;
            for (int c = -rz; c <= rz; ++c) {
                int m = k + c;
                if (m < 0 || m >= p->nz) continue;
                acc += p->gz[(size_t)m * p->kz + (c + rz)] * bl[(size_t)(m - m0) * S + q];
            }
            out[(size_t)k * S + q] = acc;
        }
    }
    free(bl);
}

void orc_H(const orc_problem *p, const double *x, double *out, int k0, int k1)
{
    if (k0 < 0) k0 = 0;
    if (k1 > p->nz) k1 = p->nz;
    if (k0 >= k1) return;
    if (p->dense || p->pk) H_dense(p, x, out, k0, k1); else H_sep(p, x, out, k0, k1);
}

void orc_HT(const orc_problem *p, const double *r, double *out, int k0, int k1)
{
    if (k0 < 0) k0 = 0;
    if (k1 > p->nz) k1 = p->nz;
    if (k0 >= k1) return;
    if (p->dense || p->pk) HT_dense(p, r, out, k0, k1); else HT_sep(p, r, out, k0, k1);
}

/* ------------------------------------------------------------------------ */
/* Discrete gradients (forward differences, last difference 0) and adjoints. */

static double dX(const orc_problem *p, const double *x, int k, int j, int i)
{
    return i < p->nx - 1 ? x[VOX(p, k, j, i + 1)] - x[VOX(p, k, j, i)] : 0.0;
}
static double dY(const orc_problem *p, const double *x, int k, int j, int i)
{
    return j < p->ny - 1 ? x[VOX(p, k, j + 1, i)] - x[VOX(p, k, j, i)] : 0.0;
}
static double dZ(const orc_problem *p, const double *x, int k, int j, int i)
{
    return k < p->nz - 1 ? x[VOX(p, k + 1, j, i)] - x[VOX(p, k, j, i)] : 0.0;
}

/* op: 0 = V^X, 1 = V^Y, 2 = V^Z; adjoint selects the transpose. */
void orc_V(const orc_problem *p, int op, int adjoint, const double *in, double *out)
{
    for (int k = 0; k < p->nz; ++k)
        for (int j = 0; j < p->ny; ++j)
            for (int i = 0; i < p->nx; ++i) {
                double v;
                if (!adjoint) {
                    v = op == 0 ? dX(p, in, k, j, i) : op == 1 ? dY(p, in, k, j, i) : dZ(p, in, k, j, i);
                } else {
                    /* (V^T q)_m = q_{m-1} [m >= 1] - q_m [m < n-1] along the axis */
                    int pos = op == 0 ? i : op == 1 ? j : k;
                    int n = op == 0 ? p->nx : op == 1 ? p->ny : p->nz;
                    v = 0.0;
                    if (pos >= 1) {
                        int ii = i - (op == 0), jj = j - (op == 1), kk = k - (op == 2);
                        v += in[VOX(p, kk, jj, ii)];
                    }
                    if (pos < n - 1) v -= in[VOX(p, k, j, i)];
                }
                out[VOX(p, k, j, i)] = v;
            }
}

static double omega_at(const orc_problem *p, const double *x, int k, int j, int i)
{
    double gxv = dX(p, x, k, j, i), gyv = dY(p, x, k, j, i);
    double gzv = p->tv3d ? dZ(p, x, k, j, i) : 0.0;
    return 1.0 / sqrt(gxv * gxv + gyv * gyv + gzv * gzv + p->delta * p->delta);
}

static double clipd(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* ------------------------------------------------------------------------ */
/* Objective and gradient (Sec. 3.1, eq. "eq_crit").                         */

/* Per-term values: terms[0] = 1/2||Hx-y||^2, [1] = eta d^2_box, [2] = lambda TV,
 * [3] = kappa ||V^Z x||^2.  Returns their sum.                              */
double orc_f_terms(const orc_problem *p, const double *x, double *terms)
{
    size_t N = nvox(p), S = nslice(p);
    double *hx = (double *)malloc(N * sizeof(double));
    double *part = (double *)calloc((size_t)4 * p->nz, sizeof(double));
    orc_H(p, x, hx, 0, p->nz);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < p->nz; ++k) {
        double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
        for (int j = 0; j < p->ny; ++j)
            for (int i = 0; i < p->nx; ++i) {
                size_t v = VOX(p, k, j, i);
                double r = hx[v] - p->y[v];
                s0 += r * r;
                double e = x[v] - clipd(x[v], p->xmin, p->xmax);
                s1 += e * e;
                double gxv = dX(p, x, k, j, i), gyv = dY(p, x, k, j, i);
                double gzv = dZ(p, x, k, j, i);
                double g3 = p->tv3d ? gzv : 0.0;
                s2 += sqrt(gxv * gxv + gyv * gyv + g3 * g3 + p->delta * p->delta);
                s3 += gzv * gzv;
            }
        part[4 * k + 0] = s0; part[4 * k + 1] = s1; part[4 * k + 2] = s2; part[4 * k + 3] = s3;
    }
    double t[4] = {0, 0, 0, 0};
    for (int k = 0; k < p->nz; ++k)
        for (int q = 0; q < 4; ++q) t[q] += part[4 * k + q];
    (void)S;
    free(hx);
    free(part);
    double out[4] = {0.5 * t[0], p->eta * t[1], p->lambda * t[2], p->kappa * t[3]};
    if (terms) memcpy(terms, out, sizeof(out));
    return out[0] + out[1] + out[2] + out[3];
}

double orc_f(const orc_problem *p, const double *x) { return orc_f_terms(p, x, NULL); }

/* grad f on slices [k0, k1) (other slices of g untouched):
 *   H^T(Hx - y) + 2 eta (x - clip x) + lambda (V^X^T(w V^X x) + V^Y^T(w V^Y x))
 *   + 2 kappa V^Z^T V^Z x.
 * Needs r = Hx - y on [k0 - rz, k1 + rz), computed here from x.             */
void orc_grad_slices(const orc_problem *p, const double *x, double *g, int k0, int k1)
{
    int rz = p->kz / 2;
    size_t N = nvox(p);
    if (k0 < 0) k0 = 0;
    if (k1 > p->nz) k1 = p->nz;
    if (k0 >= k1) return;
    int r0 = k0 - rz < 0 ? 0 : k0 - rz, r1 = k1 + rz > p->nz ? p->nz : k1 + rz;
    double *r = scratch_get(SCR_R, N);
    orc_H(p, x, r, r0, r1);
    size_t S = nslice(p);
    for (size_t q = (size_t)r0 * S; q < (size_t)r1 * S; ++q) r[q] -= p->y[q];
    orc_HT(p, r, g, k0, k1);
    scratch_clear(r, r0, r1, S);
#pragma omp parallel for schedule(static)
    for (int k = k0; k < k1; ++k)
        for (int j = 0; j < p->ny; ++j)
            for (int i = 0; i < p->nx; ++i) {
                size_t v = VOX(p, k, j, i);
                double acc = g[v];
                acc += 2.0 * p->eta * (x[v] - clipd(x[v], p->xmin, p->xmax));
                /* lambda * (V^X^T (w V^X x) + V^Y^T (w V^Y x)) at (k,j,i) */
                double tv = 0.0;
                if (i >= 1) tv += omega_at(p, x, k, j, i - 1) * dX(p, x, k, j, i - 1);
                if (i < p->nx - 1) tv -= omega_at(p, x, k, j, i) * dX(p, x, k, j, i);
                if (j >= 1) tv += omega_at(p, x, k, j - 1, i) * dY(p, x, k, j - 1, i);
                if (j < p->ny - 1) tv -= omega_at(p, x, k, j, i) * dY(p, x, k, j, i);
                if (p->tv3d) {  /* V^Z^T (w V^Z x) */
                    if (k >= 1) tv += omega_at(p, x, k - 1, j, i) * dZ(p, x, k - 1, j, i);
                    if (k < p->nz - 1) tv -= omega_at(p, x, k, j, i) * dZ(p, x, k, j, i);
                }
                acc += p->lambda * tv;
                if (p->kappa != 0.0) {
                    double zz = 0.0;
                    if (k >= 1) zz += dZ(p, x, k - 1, j, i);
                    if (k < p->nz - 1) zz -= dZ(p, x, k, j, i);
                    acc += 2.0 * p->kappa * zz;
                }
                g[v] = acc;
            }
}

void orc_grad(const orc_problem *p, const double *x, double *g)
{
    orc_grad_slices(p, x, g, 0, p->nz);
}

/* Plain dot product over slices [k0, k1), per-slice partials in order. */
static double dot_slices(const orc_problem *p, const double *a, const double *b, int k0, int k1)
{
    size_t S = nslice(p);
    if (k0 < 0) k0 = 0;
    if (k1 > p->nz) k1 = p->nz;
    if (k0 >= k1) return 0.0;
    double *part = (double *)calloc((size_t)(k1 - k0), sizeof(double));
#pragma omp parallel for schedule(static)
    for (int k = k0; k < k1; ++k) {
        double s = 0.0;
        for (size_t q = 0; q < S; ++q) s += a[(size_t)k * S + q] * b[(size_t)k * S + q];
        part[k - k0] = s;
    }
    double s = 0.0;
    for (int k = k0; k < k1; ++k) s += part[k - k0];
    free(part);
    return s;
}

double orc_dot(const orc_problem *p, const double *a, const double *b)
{
    return dot_slices(p, a, b, 0, p->nz);
}

/* ------------------------------------------------------------------------ */
/* Majorant bilinear form a(u, v) = u^T A(x) v, for u, v supported on slices
 * [z0, z1) (pass 0, nz for arbitrary u, v).                                 */
double orc_majorant_form(const orc_problem *p, const double *x, const double *u,
                         const double *v, int z0, int z1)
{
    int rz = p->kz / 2;
    size_t N = nvox(p);
    if (z0 < 0) z0 = 0;
    if (z1 > p->nz) z1 = p->nz;
    int h0 = z0 - rz < 0 ? 0 : z0 - rz, h1 = z1 + rz > p->nz ? p->nz : z1 + rz;
    double *hu = scratch_get(SCR_HU, N);
    double *hv = scratch_get(SCR_HV, N);
    orc_H(p, u, hu, h0, h1);
    orc_H(p, v, hv, h0, h1);
    double quad = dot_slices(p, hu, hv, h0, h1);
    scratch_clear(hu, h0, h1, nslice(p));
    scratch_clear(hv, h0, h1, nslice(p));
    double box = dot_slices(p, u, v, z0, z1);
    /* with 3D TV the difference along z of u, v reaches slice z0 - 1 */
    int t0 = (p->tv3d && z0 >= 1) ? z0 - 1 : z0;
    int nzs = z1 - t0;
    double *part = (double *)calloc((size_t)(nzs > 0 ? nzs : 1), sizeof(double));
#pragma omp parallel for schedule(static)
    for (int k = t0; k < z1; ++k) {
        double s = 0.0;
        for (int j = 0; j < p->ny; ++j)
            for (int i = 0; i < p->nx; ++i) {
                double w = omega_at(p, x, k, j, i);
                double d = dX(p, u, k, j, i) * dX(p, v, k, j, i) + dY(p, u, k, j, i) * dY(p, v, k, j, i);
                if (p->tv3d) d += dZ(p, u, k, j, i) * dZ(p, v, k, j, i);
                s += w * d;
            }
        part[k - t0] = s;
    }
    double tv = 0.0;
    for (int k = t0; k < z1; ++k) tv += part[k - t0];
    free(part);
    double zz = 0.0;
    if (p->kappa != 0.0) {
        int a0 = z0 - 1 < 0 ? 0 : z0 - 1;
        for (int k = a0; k < z1; ++k)
            for (int j = 0; j < p->ny; ++j)
                for (int i = 0; i < p->nx; ++i) zz += dZ(p, u, k, j, i) * dZ(p, v, k, j, i);
    }
    return quad + 2.0 * p->eta * box + p->lambda * tv + 2.0 * p->kappa * zz;
}

/* Majorant matrix applied to a block vector (Sec. 2.2, eq. "maj": the
 * half-quadratic A(x) of the criterion; A_(S) its principal submatrix on the
 * block S = [z0, z1)): for u supported on S (zero elsewhere),
 *   out_S = [H^T H u + 2 eta u + lambda (V^X^T(w V^X u) + V^Y^T(w V^Y u))
 *            + 2 kappa V^Z^T V^Z u]_S + mu u_S,   w = omega(x),
 * and out is left untouched outside S.  <v, out> equals the bilinear form
 * orc_majorant_form(u, v) (+ mu <u, v>) for v supported on S. */
void orc_majorant_apply(const orc_problem *p, const double *x, const double *u, double *out,
                        int z0, int z1)
{
    int rz = p->kz / 2;
    size_t N = nvox(p), S = nslice(p);
    if (z0 < 0) z0 = 0;
    if (z1 > p->nz) z1 = p->nz;
    if (z0 >= z1) return;
    int h0 = z0 - rz < 0 ? 0 : z0 - rz, h1 = z1 + rz > p->nz ? p->nz : z1 + rz;
    double *hu = scratch_get(SCR_HU, N);
    orc_H(p, u, hu, h0, h1);
    orc_HT(p, hu, out, z0, z1);
    scratch_clear(hu, h0, h1, S);
#pragma omp parallel for schedule(static)
    for (int k = z0; k < z1; ++k)
        for (int j = 0; j < p->ny; ++j)
            for (int i = 0; i < p->nx; ++i) {
                size_t v = VOX(p, k, j, i);
                double acc = out[v] + 2.0 * p->eta * u[v];
                double tv = 0.0;
                if (i >= 1) tv += omega_at(p, x, k, j, i - 1) * dX(p, u, k, j, i - 1);
                if (i < p->nx - 1) tv -= omega_at(p, x, k, j, i) * dX(p, u, k, j, i);
                if (j >= 1) tv += omega_at(p, x, k, j - 1, i) * dY(p, u, k, j - 1, i);
                if (j < p->ny - 1) tv -= omega_at(p, x, k, j, i) * dY(p, u, k, j, i);
                if (p->tv3d) {
                    if (k >= 1) tv += omega_at(p, x, k - 1, j, i) * dZ(p, u, k - 1, j, i);
                    if (k < p->nz - 1) tv -= omega_at(p, x, k, j, i) * dZ(p, u, k, j, i);
                }
                acc += p->lambda * tv;
                if (p->kappa != 0.0) {
                    double zz = 0.0;
                    if (k >= 1) zz += dZ(p, u, k - 1, j, i);
                    if (k < p->nz - 1) zz -= dZ(p, u, k, j, i);
                    acc += 2.0 * p->kappa * zz;
                }
                out[v] = acc + p->mu * u[v];
            }
}

/* ------------------------------------------------------------------------ */
/* Moore-Penrose inverse of the symmetric PSD 2x2 matrix [[b11, b12],[b12, b22]]
 * (Sec. 2.3, eq. "minimizer").  Full rank when det > 1e-12 b11 b22: exact
 * inverse.  Otherwise treated as rank one, B = v v^T, whose pseudo-inverse is
 * B / tr(B)^2; zero when tr(B) = 0.  B in: {b11, b12, b22}; out: same layout. */
void orc_pinv2(const double *B, double *P)
{
    double b11 = B[0], b12 = B[1], b22 = B[2];
    double det = b11 * b22 - b12 * b12;
    double tr = b11 + b22;
    if (det > 1e-12 * b11 * b22) {
        P[0] = b22 / det;
        P[1] = -b12 / det;
        P[2] = b11 / det;
    } else if (tr > 0.0) {
        double t2 = tr * tr;
        P[0] = b11 / t2;
        P[1] = b12 / t2;
        P[2] = b22 / t2;
    } else {
        P[0] = P[1] = P[2] = 0.0;
    }
}

/* ------------------------------------------------------------------------ */
/* Block colouring used to order the sweep: blocks in z order; block b takes
 * the smallest colour none of whose earlier members lies closer than
 * min_gap slices (slices strictly between the two blocks).  Same-colour
 * blocks then touch disjoint parts of the state, so updating them in any
 * order gives the same iterate as the sequential rule of Sec. 3.1.  The
 * sweep order is colours ascending, z ascending within a colour.
 * Returns the number of colours; order[] receives the block indices.       */
int orc_color_schedule(int nblocks, const int *nslices, int min_gap, int *order, int *color)
{
    int *z0 = (int *)malloc((size_t)nblocks * sizeof(int));
    int z = 0, ncol = 0;
    for (int b = 0; b < nblocks; ++b) { z0[b] = z; z += nslices[b]; }
    for (int b = 0; b < nblocks; ++b) {
        int c = 0;
        for (;; ++c) {
            int ok = 1;
            for (int e = 0; e < b; ++e) {
                if (color[e] != c) continue;
                int gap = z0[b] - (z0[e] + nslices[e]);
                if (gap < min_gap) { ok = 0; break; }
            }
            if (ok) break;
        }
        color[b] = c;
        if (c + 1 > ncol) ncol = c + 1;
    }
    int q = 0;
    for (int c = 0; c < ncol; ++c)
        for (int b = 0; b < nblocks; ++b)
            if (color[b] == c) order[q++] = b;
    free(z0);
    return ncol;
}

/* ------------------------------------------------------------------------ */
/* One worker step (box "Worker" of Sec. 2.3) on the block of slices
 * [z0, z0 + n), followed by the Master's update x_S += d'.
 *   x      : iterate, updated in place on S;
 *   dprev  : full-size volume holding each block's previous step on its own
 *            slices; updated in place on S;
 *   info   : optional, receives {B11, B12, B22, c1, c2, u1, u2, ||g||^2}.   */
/* One block's memory-gradient MM step at the point x (Sec. 2.3, box "Worker";
 * eq. "minimizer"): g = grad f(x) on S, D = [-g | d_prev], B = D^T A_S(x) D
 * with A_S the principal submatrix of the majorant, plus mu Id when the
 * problem's mu > 0 (the curvature inflation of Assumption C), u = -B^+ D^T g,
 * d' = D u.
 * d' is written to dout on S only; x and dprev are not changed. */
/* Async-MM's inner solve (Sec. 3.2: the Worker's direction becomes
 * d' = -A_(S)(x)^{-1} grad_S f(x), the inversion done by a linear biconjugate
 * gradient solver): BiCG on A_S(x) v = b, b = -g_S, from v = 0, with the
 * shadow residual started at the residual.  At most n_inner iterations;
 * stops early when ||r_k|| <= tol_inner ||r_0|| or when <rt, r> or
 * <pt, A p> vanishes.  v (on S) is written to vout; returns the iterations
 * done and stores ||r||^2 at the end in *rr_end. */
static int bicg_block(const orc_problem *p, const double *x, const double *g, double *vout, int z0, int n,
                      double *rr_end)
{
    size_t N = nvox(p), S = nslice(p);
    size_t off = (size_t)z0 * S, cnt = (size_t)n * S;
    int z1 = z0 + n;
    double *r = (double *)calloc(N, sizeof(double));
    double *rt = (double *)calloc(N, sizeof(double));
    double *pv = (double *)calloc(N, sizeof(double));
    double *pt = (double *)calloc(N, sizeof(double));
    double *ap = (double *)calloc(N, sizeof(double));
    double *apt = (double *)calloc(N, sizeof(double));
    for (size_t q = off; q < off + cnt; ++q) {
        vout[q] = 0.0;
        r[q] = -g[q];  /* r_0 = b - A v_0, v_0 = 0 */
        rt[q] = r[q];
        pv[q] = r[q];
        pt[q] = rt[q];
    }
    double r0 = sqrt(dot_slices(p, r, r, z0, z1));
    double rho = dot_slices(p, rt, r, z0, z1);
    int it = 0;
    while (it < p->n_inner && rho != 0.0) {
        orc_majorant_apply(p, x, pv, ap, z0, z1);
        /* A_S(x) is symmetric, so the shadow system's A^T pt is A pt */
        orc_majorant_apply(p, x, pt, apt, z0, z1);
        double den = dot_slices(p, pt, ap, z0, z1);
        if (den == 0.0) break;
        double alpha = rho / den;
        for (size_t q = off; q < off + cnt; ++q) {
            vout[q] += alpha * pv[q];
            r[q] -= alpha * ap[q];
            rt[q] -= alpha * apt[q];
        }
        ++it;
        if (p->tol_inner > 0.0 && sqrt(dot_slices(p, r, r, z0, z1)) <= p->tol_inner * r0) break;
        double rho1 = dot_slices(p, rt, r, z0, z1);
        double beta = rho1 / rho;
        rho = rho1;
        for (size_t q = off; q < off + cnt; ++q) {
            pv[q] = r[q] + beta * pv[q];
            pt[q] = rt[q] + beta * pt[q];
        }
    }
    if (rr_end) *rr_end = dot_slices(p, r, r, z0, z1);
    free(r); free(rt); free(pv); free(pt); free(ap); free(apt);
    return it;
}

/* The Worker's direction for the ablation variants of Sec. 3.2 (p->method
 * 1-3), from the gradient g on S; d' to dout on S.  info as for BD3MG:
 * GD and CG give {B11, B12, B22, c1, c2, u1, u2, ||g||^2} of their metric
 * L Id (GD: B12 = B22 = c2 = u2 = 0); MM gives {iterations, ||r_end||^2,
 * 0, c1, 0, 0, 0, ||g||^2}. */
static void ablation_direction(const orc_problem *p, const double *x, const double *dprev, const double *g,
                               int z0, int n, double *dout, double *info)
{
    size_t S = nslice(p);
    size_t off = (size_t)z0 * S, cnt = (size_t)n * S;
    int z1 = z0 + n;
    double gg = dot_slices(p, g, g, z0, z1);
    double lm = p->lip + p->mu;
    double B[3] = {0, 0, 0}, c1 = -gg, c2 = 0.0, u1 = 0.0, u2 = 0.0;
    if (p->method == 1) {
        /* D = [-g], A_S = L Id: B = L <g, g>, c = <-g, g>, u = -B^+ c */
        B[0] = lm * gg;
        u1 = B[0] > 0.0 ? -c1 / B[0] : 0.0;
        for (size_t q = off; q < off + cnt; ++q) dout[q] = u1 * -g[q];
    } else if (p->method == 2) {
        /* BD3MG's Worker step with the basic metric A_S = L Id: D = [-g, d],
         * B = L D^T D, c = D^T g, u = -B^+ c.  Since -g lies in the range of
         * D, D u = -g / L: the step of Async-GD, up to rounding. */
        double gd = dot_slices(p, g, dprev, z0, z1), dd = dot_slices(p, dprev, dprev, z0, z1);
        B[0] = lm * gg;
        B[1] = -lm * gd;
        B[2] = lm * dd;
        c2 = gd;
        double P[3];
        orc_pinv2(B, P);
        u1 = -(P[0] * c1 + P[1] * c2);
        u2 = -(P[1] * c1 + P[2] * c2);
        for (size_t q = off; q < off + cnt; ++q) dout[q] = u1 * -g[q] + u2 * dprev[q];
    } else {
        double rr = 0.0;
        int it = bicg_block(p, x, g, dout, z0, n, &rr);
        B[0] = (double)it;
        B[1] = rr;
    }
    if (info) {
        info[0] = B[0]; info[1] = B[1]; info[2] = B[2];
        info[3] = c1; info[4] = c2; info[5] = u1; info[6] = u2;
        info[7] = gg;
    }
}

static void block_direction(const orc_problem *p, const double *x, const double *dprev, int z0, int n,
                            double *dout, double *info)
{
    size_t N = nvox(p), S = nslice(p);
    if (p->method != 0) {
        double *ga = scratch_get(SCR_G, N);
        orc_grad_slices(p, x, ga, z0, z0 + n);
        ablation_direction(p, x, dprev, ga, z0, n, dout, info);
        scratch_clear(ga, z0, z0 + n, S);
        return;
    }
    size_t off = (size_t)z0 * S, cnt = (size_t)n * S;
    double *g = scratch_get(SCR_G, N);
    double *d1 = scratch_get(SCR_D1, N);
    double *d2 = scratch_get(SCR_D2, N);
    /* gradient on the block, subspace directions [-g | d] */
    orc_grad_slices(p, x, g, z0, z0 + n);
    for (size_t q = off; q < off + cnt; ++q) {
        d1[q] = -g[q];
        d2[q] = dprev[q];
    }
    /* D^T A_S D and D^T grad */
    double B[3];
    B[0] = orc_majorant_form(p, x, d1, d1, z0, z0 + n);
    B[1] = orc_majorant_form(p, x, d1, d2, z0, z0 + n);
    B[2] = orc_majorant_form(p, x, d2, d2, z0, z0 + n);
    if (p->mu > 0.0) {
        B[0] += p->mu * dot_slices(p, d1, d1, z0, z0 + n);
        B[1] += p->mu * dot_slices(p, d1, d2, z0, z0 + n);
        B[2] += p->mu * dot_slices(p, d2, d2, z0, z0 + n);
    }
    double c1 = dot_slices(p, d1, g, z0, z0 + n);
    double c2 = dot_slices(p, d2, g, z0, z0 + n);
    double P[3];
    orc_pinv2(B, P);
    /* u = -(D^T A D)^+ D^T grad, d' = D u */
    double u1 = -(P[0] * c1 + P[1] * c2);
    double u2 = -(P[1] * c1 + P[2] * c2);
    for (size_t q = off; q < off + cnt; ++q) dout[q] = u1 * d1[q] + u2 * d2[q];
    if (info) {
        info[0] = B[0]; info[1] = B[1]; info[2] = B[2];
        info[3] = c1; info[4] = c2; info[5] = u1; info[6] = u2;
        info[7] = -c1;
    }
    scratch_clear(g, z0, z0 + n, S);
    scratch_clear(d1, z0, z0 + n, S);
    scratch_clear(d2, z0, z0 + n, S);
}

/* Block update without delay: the step of block [z0, z0+n) at the current x,
 * applied at once (x += d', d_prev = d' on the block). */
void orc_block_step(const orc_problem *p, double *x, double *dprev, int z0, int n, double *info)
{
    size_t N = nvox(p), S = nslice(p);
    size_t off = (size_t)z0 * S, cnt = (size_t)n * S;
    double *dn = scratch_get(SCR_DN, N);
    block_direction(p, x, dprev, z0, n, dn, info);
    for (size_t q = off; q < off + cnt; ++q) {
        x[q] += dn[q];
        dprev[q] = dn[q];
    }
    scratch_clear(dn, z0, z0 + n, S);
}

static double norm_grad(const orc_problem *p, const double *x)
{
    size_t N = nvox(p);
    double *g = (double *)malloc(N * sizeof(double));
    orc_grad(p, x, g);
    double s = sqrt(orc_dot(p, g, g));
    free(g);
    return s;
}

double orc_grad_norm(const orc_problem *p, const double *x) { return norm_grad(p, x); }

/* Asynchronous rounds (Sec. 2.4-2.5): every block computes its step from the
 * same snapshot x^k (the delays of a round are at most tau = nblocks - 1
 * block updates, Assumption B), then all steps are applied.  The problem's mu
 * inflates each block's majorant by mu Id (Assumption C).  Stops as orc_run
 * does. */
int orc_run_round(const orc_problem *p, double *x, double *dprev, int nblocks, const int *nslices,
                  int max_sweeps, double grad_rtol, double gnorm_ref, double *f_hist, double *g_hist)
{
    size_t N = nvox(p);
    double *dn = (double *)calloc(N, sizeof(double));
    int s;
    for (s = 0; s < max_sweeps; ++s) {
        int z0 = 0;
        for (int b = 0; b < nblocks; ++b) {
            block_direction(p, x, dprev, z0, nslices[b], dn, NULL);
            z0 += nslices[b];
        }
        for (size_t q = 0; q < N; ++q) {
            x[q] += dn[q];
            dprev[q] = dn[q];
        }
        double gn = -1.0;
        if (f_hist) f_hist[s] = orc_f(p, x);
        if (g_hist || grad_rtol > 0.0) gn = norm_grad(p, x);
        if (g_hist) g_hist[s] = gn;
        if (grad_rtol > 0.0 && gn <= grad_rtol * gnorm_ref) { ++s; break; }
    }
    free(dn);
    return s;
}

/* A Lipschitz constant of grad f (Assumption A) bounded from the tables:
 * ||H^T H|| <= ||H||_1 ||H||_inf (H >= 0, the in-slice factors sum to 1, so
 * the row sums are the z weights of the output slice and the column sums
 * those gathered from the slices an input slice reaches), plus 2 eta for the
 * box term, lambda ||D||^2 / delta with ||D||^2 <= 8 for the two in-slice
 * forward differences (omega <= 1 / delta), and 2 kappa ||V^Z||^2 <= 8 kappa. */
double orc_lipschitz_bound(const orc_problem *p)
{
    int rz = p->kz / 2;
    /* ||[V^X; V^Y]||^2 <= 8, and 12 with V^Z inside the root as well (each
     * forward difference has norm <= 2); omega <= 1 / delta */
    double tvc = p->tv3d ? 12.0 : 8.0;
    double rmax = 0.0, cmax = 0.0;
    if (p->pk) {
        /* general kernels: row sums of |H| are bounded by sum |P_k| of the
         * output slice, column sums by what an input slice s gathers from the
         * slices s + c it reaches, sum_c sum_{b,a} |P_{s+c}[c][b][a]| */
        size_t kk = (size_t)p->ky * p->kx;
        for (int k = 0; k < p->nz; ++k) {
            double r = 0.0, c = 0.0;
            for (int t = -rz; t <= rz; ++t)
                for (size_t q = 0; q < kk; ++q) {
                    r += fabs(p->pk[((size_t)k * p->kz + t + rz) * kk + q]);
                    if (k + t >= 0 && k + t < p->nz) c += fabs(p->pk[((size_t)(k + t) * p->kz + t + rz) * kk + q]);
                }
            if (r > rmax) rmax = r;
            if (c > cmax) cmax = c;
        }
        return rmax * cmax + 2.0 * p->eta + tvc * p->lambda / p->delta + 8.0 * p->kappa;
    }
    for (int k = 0; k < p->nz; ++k) {
        double r = 0.0, c = 0.0;
        for (int t = -rz; t <= rz; ++t) {
            if (k - t >= 0 && k - t < p->nz) r += fabs(p->gz[(size_t)k * p->kz + t + rz]);
            if (k + t >= 0 && k + t < p->nz) c += fabs(p->gz[(size_t)(k + t) * p->kz + t + rz]);
        }
        if (r > rmax) rmax = r;
        if (c > cmax) cmax = c;
    }
    double sx = 0.0, sy = 0.0;
    for (int k = 0; k < p->nz; ++k) {
        double ax = 0.0, ay = 0.0;
        for (int a = 0; a < p->kx; ++a) ax += fabs(p->gx[(size_t)k * p->kx + a]);
        for (int a = 0; a < p->ky; ++a) ay += fabs(p->gy[(size_t)k * p->ky + a]);
        if (ax > sx) sx = ax;
        if (ay > sy) sy = ay;
    }
    double hh = rmax * cmax * sx * sx * sy * sy;
    return hh + 2.0 * p->eta + tvc * p->lambda / p->delta + 8.0 * p->kappa;
}

/* ------------------------------------------------------------------------ */
/* BD3MG driver with no delay (delta_k = 0, Sec. 2.4): blocks are visited in
 * order[] (a permutation of 0..nblocks-1), one sweep = every block once.
 * After each sweep, f and ||grad f|| are recorded when the histories are
 * given.  Stops after max_sweeps, or once ||grad f(x)|| <= grad_rtol *
 * gnorm_ref (grad_rtol > 0; checked after every sweep).  Returns the number
 * of sweeps done.  x and dprev are the state and are updated in place, so a
 * run can be resumed.                                                       */
int orc_run(const orc_problem *p, double *x, double *dprev, int nblocks, const int *nslices,
            const int *order, int max_sweeps, double grad_rtol, double gnorm_ref,
            double *f_hist, double *g_hist)
{
    int *z0 = (int *)malloc((size_t)nblocks * sizeof(int));
    int z = 0;
    for (int b = 0; b < nblocks; ++b) { z0[b] = z; z += nslices[b]; }
    int s;
    for (s = 0; s < max_sweeps; ++s) {
        for (int q = 0; q < nblocks; ++q) {
            int b = order[q];
            orc_block_step(p, x, dprev, z0[b], nslices[b], NULL);
        }
        double gn = -1.0;
        if (f_hist) f_hist[s] = orc_f(p, x);
        if (g_hist || grad_rtol > 0.0) gn = norm_grad(p, x);
        if (g_hist) g_hist[s] = gn;
        if (grad_rtol > 0.0 && gn <= grad_rtol * gnorm_ref) { ++s; break; }
    }
    free(z0);
    return s;
}
