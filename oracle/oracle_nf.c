/*
 * oracle_nf.c -- plain FP64 CPU oracle for the Abacus near-field force.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline of the benchmark may load this library.  It shares no code,
 * header, table or constant with the HIP path.
 *
 * What it computes (Sec. 3.1 "Force Solver Algorithm and Serial Method"):
 * the box is periodic and cut into K^3 cubic cells; the near field of a sink
 * particle is every particle in the cells within R cells of the sink's cell
 * (R=2 gives the 5x5x5 block), each taken at the periodic image that lies in
 * that neighbouring cell -- images are explicit, there is no minimum-image or
 * non-periodic approximation of close pairs.  The near-field acceleration is
 * the direct O(N^2) sum over that set:
 *
 *     a_i = G*m * sum_{(j,s) in NF(i)} d * g(|d|),   d = (x_j + s*L) - x_i
 *
 * with g the softened inverse cube (attractive: d points from i to j).
 *
 * Softening laws (Sec. 2.5 "Code Parameters" and Sec. 5.2 "Accuracy"):
 *   kind 0, spline : g = 1/r^3 for r >= eps (exact Newtonian force beyond a
 *                    finite radius); inside, the force is the cubic
 *                    polynomial in r that matches the value, slope and
 *                    curvature of 1/r^2 at r = eps:
 *                    F(r)*eps^2 = 10u - 15u^2 + 6u^3, u = r/eps,
 *                    i.e. g = (10 - 15u + 6u^2)/eps^3.  The paper does not
 *                    print this polynomial (it cites a companion paper); the
 *                    matching conditions are the reading used here.
 *   kind 1, Plummer: potential -1/sqrt(r^2+eps^2), so g = (r^2+eps^2)^(-3/2).
 *
 * Cell rule (the paper is silent; reading): with xt = x - L*floor(x/L) and
 * s = K/L, the cell index along an axis is c = min(floor(xt*s), K-1), all in
 * FP64 from the FP32 input, each operation rounded separately (no fused
 * multiply-add; build with -ffp-contract=off).  Linear cell index
 * (cx*K + cy)*K + cz.
 *
 * Kernel density estimate (Sec. 3.3 "Halo Finding"): computed in the same
 * near-field pass, the density of particle i is the sum over its near field
 * of the weight max(0, 1 - r^2/b^2) (b is a fixed radius; the paper takes 40%
 * of the mean interparticle spacing).  The self pair is included (weight 1):
 * the paper does not say, and this is the reading used here.
 *
 * Cell multipoles (Sec. 3.1: the far field starts from the multipole moments
 * of the mass in each cell, order p = 8): complete Cartesian moments about the
 * cell centre in cell widths (see oracle_nf_multipoles).
 *
 * Far field from per-cell Taylor series (Sec. 3.1): the gradient of
 * Phi = sum T^(a,b,k) u^a v^b w^k about each cell centre, added to a force
 * array (see oracle_nf_taylor).
 *
 * Coincident particles (including the self pair) contribute exactly zero force.
 * Sums are plain FP64 in a fixed order (neighbour cells in lexicographic
 * (dx,dy,dz) order, sources in input order within a cell), or Neumaier
 * compensated FP64 when requested, as a self-check of the oracle's own
 * rounding.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_EINVAL -1
#define ORACLE_ENOMEM -2

/* Axis cell index and wrapped coordinate, per the cell rule above. */
static inline int axis_cell(double x, double L, double s, int K, double *xt_out) {
    double q = floor(x / L);
    double xt = x - L * q;
    double t = xt * s;
    double f = floor(t);
    int c = (f >= (double)(K - 1)) ? (K - 1) : (int)f;
    if (c < 0) c = 0;
    *xt_out = xt;
    return c;
}

/* Exported for the tests: the cell of every particle (linear index). */
int oracle_nf_bin(const float *pos, int64_t n, double L, int K, int32_t *cell_out) {
    if (n < 0 || !(L > 0) || K < 1 || (n > 0 && (!pos || !cell_out))) return ORACLE_EINVAL;
    double s = (double)K / L;
    for (int64_t i = 0; i < n; i++) {
        double xt;
        int cx = axis_cell((double)pos[3 * i + 0], L, s, K, &xt);
        int cy = axis_cell((double)pos[3 * i + 1], L, s, K, &xt);
        int cz = axis_cell((double)pos[3 * i + 2], L, s, K, &xt);
        cell_out[i] = (int32_t)(((int64_t)cx * K + cy) * K + cz);
    }
    return ORACLE_OK;
}

/* The softened inverse cube g(r) given r^2 > 0. */
static inline double kernel_g(double r2, double eps, int kind) {
    if (kind == 1) {
        double q = r2 + eps * eps;
        return 1.0 / (q * sqrt(q));
    }
    double r = sqrt(r2);
    if (r >= eps) return 1.0 / (r2 * r);
    double u = r / eps;
    return (10.0 - 15.0 * u + 6.0 * u * u) / (eps * eps * eps);
}

/* Exported for the tests: g(r) on an array of separations. */
int oracle_nf_kernel(const double *r, int64_t n, double eps, int kind, double *g_out) {
    if (n < 0 || !(eps > 0) || (kind != 0 && kind != 1)) return ORACLE_EINVAL;
    for (int64_t i = 0; i < n; i++) g_out[i] = (r[i] > 0) ? kernel_g(r[i] * r[i], eps, kind) : 0.0;
    return ORACLE_OK;
}

typedef struct {
    double s0, c0, s1, c1, s2, c2;  /* running sums and Neumaier compensations */
} acc3;

static inline void neumaier_add(double *s, double *c, double v) {
    double t = *s + v;
    if (fabs(*s) >= fabs(v)) *c += (*s - t) + v;
    else *c += (v - t) + *s;
    *s = t;
}

/*
 * Near-field accelerations for the sinks listed in `sinks` (or every particle
 * when sinks == NULL), one periodic box.
 *   pos   [n][3] float32, any finite values (wrapped into [0,L) by the cell rule)
 *   acc   [nsinks][3] float64 out, in the order of `sinks`
 *   mag   [nsinks] float64 out or NULL: G*m * sum over the near field of the
 *         magnitude of each pair term, |d| g(|d|) (the scale of the rounding
 *         error any summation order of those terms can make)
 *   pairs total number of (sink, source) pairs visited, self pair included
 * Returns 0, or a negative code for bad arguments / allocation failure.
 */
int oracle_nf_forces(const float *pos, int64_t n, double L, int K, int R, double eps, int kind,
                     double gm, const int64_t *sinks, int64_t nsinks, int neumaier, int nthreads,
                     double *acc, double *mag, int64_t *pairs) {
    if (n < 0 || !(L > 0) || R < 1 || K < 2 * R + 1 || !(eps > 0) || (kind != 0 && kind != 1))
        return ORACLE_EINVAL;
    if (sinks == NULL) nsinks = n;
    if (nsinks < 0 || (nsinks > 0 && (!acc || !pos))) return ORACLE_EINVAL;
    if (pairs) *pairs = 0;
    if (nsinks == 0) return ORACLE_OK;
    int64_t ncell = (int64_t)K * K * K;
    double s = (double)K / L;
    int32_t *cell = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    double *xt = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    int64_t *start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    int64_t *list = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)ncell);
    if (!cell || !xt || !start || !list || !fill) {
        free(cell); free(xt); free(start); free(list); free(fill);
        return ORACLE_ENOMEM;
    }
    /* bin every particle; keep its wrapped FP64 coordinates */
    for (int64_t i = 0; i < n; i++) {
        int c3[3];
        for (int d = 0; d < 3; d++) c3[d] = axis_cell((double)pos[3 * i + d], L, s, K, &xt[3 * i + d]);
        cell[i] = (int32_t)(((int64_t)c3[0] * K + c3[1]) * K + c3[2]);
    }
    /* counting sort: per-cell lists in increasing input index */
    for (int64_t i = 0; i < n; i++) start[cell[i] + 1]++;
    for (int64_t c = 0; c < ncell; c++) start[c + 1] += start[c];
    memcpy(fill, start, sizeof(int64_t) * (size_t)ncell);
    for (int64_t i = 0; i < n; i++) list[fill[cell[i]]++] = i;

    int64_t total_pairs = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : total_pairs)
#endif
    for (int64_t q = 0; q < nsinks; q++) {
        int64_t i = sinks ? sinks[q] : q;
        if (i < 0 || i >= n) {  /* out-of-range sink: report NaN */
            acc[3 * q] = acc[3 * q + 1] = acc[3 * q + 2] = NAN;
            if (mag) mag[q] = NAN;
            continue;
        }
        int ci = cell[i];
        int cz = ci % K, cy = (ci / K) % K, cx = ci / (K * K);
        double xi = xt[3 * i], yi = xt[3 * i + 1], zi = xt[3 * i + 2];
        acc3 a = {0, 0, 0, 0, 0, 0};
        double m = 0.0;
        for (int dx = -R; dx <= R; dx++) {
            int ex = cx + dx, sx = 0;
            if (ex < 0) { ex += K; sx = -1; } else if (ex >= K) { ex -= K; sx = 1; }
            for (int dy = -R; dy <= R; dy++) {
                int ey = cy + dy, sy = 0;
                if (ey < 0) { ey += K; sy = -1; } else if (ey >= K) { ey -= K; sy = 1; }
                for (int dz = -R; dz <= R; dz++) {
                    int ez = cz + dz, sz = 0;
                    if (ez < 0) { ez += K; sz = -1; } else if (ez >= K) { ez -= K; sz = 1; }
                    int64_t cj = ((int64_t)ex * K + ey) * K + ez;
                    for (int64_t k = start[cj]; k < start[cj + 1]; k++) {
                        int64_t j = list[k];
                        double ddx = (xt[3 * j] + sx * L) - xi;
                        double ddy = (xt[3 * j + 1] + sy * L) - yi;
                        double ddz = (xt[3 * j + 2] + sz * L) - zi;
                        double r2 = ddx * ddx + ddy * ddy + ddz * ddz;
                        total_pairs++;
                        if (r2 == 0.0) continue;
                        double g = kernel_g(r2, eps, kind);
                        if (mag) m += sqrt(r2) * g;
                        if (neumaier) {
                            neumaier_add(&a.s0, &a.c0, ddx * g);
                            neumaier_add(&a.s1, &a.c1, ddy * g);
                            neumaier_add(&a.s2, &a.c2, ddz * g);
                        } else {
                            a.s0 += ddx * g;
                            a.s1 += ddy * g;
                            a.s2 += ddz * g;
                        }
                    }
                }
            }
        }
        acc[3 * q + 0] = gm * (a.s0 + a.c0);
        acc[3 * q + 1] = gm * (a.s1 + a.c1);
        acc[3 * q + 2] = gm * (a.s2 + a.c2);
        if (mag) mag[q] = gm * m;
    }
    if (pairs) *pairs = total_pairs;
    free(cell); free(xt); free(start); free(list); free(fill);
    return ORACLE_OK;
}

/* Exact pair count sum_c n_c * sum_{c' in N(c)} n_c' from occupancy alone. */
int oracle_nf_count_pairs(const float *pos, int64_t n, double L, int K, int R, int64_t *pairs) {
    if (n < 0 || !(L > 0) || R < 1 || K < 2 * R + 1 || !pairs) return ORACLE_EINVAL;
    int64_t ncell = (int64_t)K * K * K;
    int64_t *cnt = (int64_t *)calloc((size_t)ncell, sizeof(int64_t));
    int32_t *cell = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!cnt || !cell) { free(cnt); free(cell); return ORACLE_ENOMEM; }
    oracle_nf_bin(pos, n, L, K, cell);
    for (int64_t i = 0; i < n; i++) cnt[cell[i]]++;
    int64_t total = 0;
    for (int64_t c = 0; c < ncell; c++) {
        if (!cnt[c]) continue;
        int cz = (int)(c % K), cy = (int)((c / K) % K), cx = (int)(c / ((int64_t)K * K));
        int64_t ns = 0;
        for (int dx = -R; dx <= R; dx++)
            for (int dy = -R; dy <= R; dy++)
                for (int dz = -R; dz <= R; dz++) {
                    int ex = ((cx + dx) % K + K) % K, ey = ((cy + dy) % K + K) % K, ez = ((cz + dz) % K + K) % K;
                    ns += cnt[((int64_t)ex * K + ey) * K + ez];
                }
        total += cnt[c] * ns;
    }
    *pairs = total;
    free(cnt); free(cell);
    return ORACLE_OK;
}

/*
 * Kernel density estimate over the near field (Sec. 3.3): for each sink,
 * rho = sum over (j, image) in NF(i) of max(0, 1 - r^2/b^2), self pair included.
 *   rho [nsinks] float64 out, in the order of `sinks` (all particles if NULL).
 * b must be positive; pairs beyond R cells are not visited, so b should not
 * exceed R cell widths for the estimate to see every neighbour within b.
 */
int oracle_nf_density(const float *pos, int64_t n, double L, int K, int R, double b, const int64_t *sinks,
                      int64_t nsinks, int nthreads, double *rho) {
    if (n < 0 || !(L > 0) || R < 1 || K < 2 * R + 1 || !(b > 0)) return ORACLE_EINVAL;
    if (sinks == NULL) nsinks = n;
    if (nsinks < 0 || (nsinks > 0 && (!rho || !pos))) return ORACLE_EINVAL;
    if (nsinks == 0) return ORACLE_OK;
    int64_t ncell = (int64_t)K * K * K;
    double s = (double)K / L;
    int32_t *cell = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    double *xt = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    int64_t *start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    int64_t *list = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)ncell);
    if (!cell || !xt || !start || !list || !fill) {
        free(cell); free(xt); free(start); free(list); free(fill);
        return ORACLE_ENOMEM;
    }
    for (int64_t i = 0; i < n; i++) {
        int c3[3];
        for (int d = 0; d < 3; d++) c3[d] = axis_cell((double)pos[3 * i + d], L, s, K, &xt[3 * i + d]);
        cell[i] = (int32_t)(((int64_t)c3[0] * K + c3[1]) * K + c3[2]);
    }
    for (int64_t i = 0; i < n; i++) start[cell[i] + 1]++;
    for (int64_t c = 0; c < ncell; c++) start[c + 1] += start[c];
    memcpy(fill, start, sizeof(int64_t) * (size_t)ncell);
    for (int64_t i = 0; i < n; i++) list[fill[cell[i]]++] = i;
    const double b2 = b * b;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t q = 0; q < nsinks; q++) {
        int64_t i = sinks ? sinks[q] : q;
        if (i < 0 || i >= n) {
            rho[q] = NAN;
            continue;
        }
        int ci = cell[i];
        int cz = ci % K, cy = (ci / K) % K, cx = ci / (K * K);
        double xi = xt[3 * i], yi = xt[3 * i + 1], zi = xt[3 * i + 2];
        double sum = 0.0;
        for (int dx = -R; dx <= R; dx++) {
            int ex = cx + dx, sx = 0;
            if (ex < 0) { ex += K; sx = -1; } else if (ex >= K) { ex -= K; sx = 1; }
            for (int dy = -R; dy <= R; dy++) {
                int ey = cy + dy, sy = 0;
                if (ey < 0) { ey += K; sy = -1; } else if (ey >= K) { ey -= K; sy = 1; }
                for (int dz = -R; dz <= R; dz++) {
                    int ez = cz + dz, sz = 0;
                    if (ez < 0) { ez += K; sz = -1; } else if (ez >= K) { ez -= K; sz = 1; }
                    int64_t cj = ((int64_t)ex * K + ey) * K + ez;
                    for (int64_t k = start[cj]; k < start[cj + 1]; k++) {
                        int64_t j = list[k];
                        double ddx = (xt[3 * j] + sx * L) - xi;
                        double ddy = (xt[3 * j + 1] + sy * L) - yi;
                        double ddz = (xt[3 * j + 2] + sz * L) - zi;
                        double w = 1.0 - (ddx * ddx + ddy * ddy + ddz * ddz) / b2;
                        if (w > 0.0) sum += w;
                    }
                }
            }
        }
        rho[q] = sum;
    }
    free(cell); free(xt); free(start); free(list); free(fill);
    return ORACLE_OK;
}

/*
 * Cell multipole moments (Sec. 3.1: the far field is built from the multipole
 * moments of the mass in each cell, order p = 8 for AbacusSummit).  Reading:
 * the complete Cartesian moments about the cell centre, in cell widths,
 *     M_c^{(a,b,k)} = m * sum_{j in c} u_j^a v_j^b w_j^k,   a + b + k <= p,
 * with (u, v, w) = (xt*K/L - (c + 1/2)) per axis, the position relative to the
 * centre of its cell in cell widths (FP64 from the FP32 input).  Components are
 * ordered by degree n = 0..p, then a = n..0, then b = n-a..0 (k = n-a-b).
 *   out [K^3][ncomp] float64, ncomp = (p+1)(p+2)(p+3)/6.
 */
int oracle_nf_multipoles(const float *pos, int64_t n, double L, int K, int p, double m, double *out) {
    if (n < 0 || !(L > 0) || K < 1 || p < 0 || p > 16 || (n > 0 && !pos) || !out) return ORACLE_EINVAL;
    const int64_t ncell = (int64_t)K * K * K;
    const int ncomp = (p + 1) * (p + 2) * (p + 3) / 6;
    const double s = (double)K / L;
    memset(out, 0, sizeof(double) * (size_t)ncell * (size_t)ncomp);
    double pu[17], pv[17], pw[17];
    for (int64_t i = 0; i < n; i++) {
        double t[3];
        int c[3];
        for (int d = 0; d < 3; d++) {
            double xt;
            c[d] = axis_cell((double)pos[3 * i + d], L, s, K, &xt);
            t[d] = xt * s - ((double)c[d] + 0.5);
        }
        pu[0] = pv[0] = pw[0] = 1.0;
        for (int q = 1; q <= p; q++) {
            pu[q] = pu[q - 1] * t[0];
            pv[q] = pv[q - 1] * t[1];
            pw[q] = pw[q - 1] * t[2];
        }
        double *o = out + (((int64_t)c[0] * K + c[1]) * K + c[2]) * ncomp;
        int idx = 0;
        for (int deg = 0; deg <= p; deg++)
            for (int a = deg; a >= 0; a--)
                for (int b = deg - a; b >= 0; b--) {
                    const int k = deg - a - b;
                    o[idx++] += m * (pu[a] * pv[b] * pw[k]);
                }
    }
    return ORACLE_OK;
}

/*
 * Far-field force from per-cell Taylor series, co-added to the near field
 * (Sec. 3.1: the far-field acceleration is a Taylor expansion of the potential
 * about each cell centre, order p; singlestep evaluates its gradient at every
 * particle and adds it to the near-field force).  With (u, v, w) the
 * particle's position relative to its cell centre in cell widths and
 *     Phi(u, v, w) = sum_{a+b+k <= p} T^(a,b,k) u^a v^b w^k
 * (coefficients in the component order of oracle_nf_multipoles), the far-field
 * acceleration in box units is -grad_x Phi = -(K/L) grad_u Phi:
 *     a_x = -(K/L) sum a T^(a,b,k) u^(a-1) v^b w^k, and likewise for y, z.
 *   taylor [K^3][ncomp] float64;  acc [n][3] float64 in/out (the far field is added).
 */
int oracle_nf_taylor(const float *pos, int64_t n, double L, int K, int p, const double *taylor, double *acc) {
    if (n < 0 || !(L > 0) || K < 1 || p < 0 || p > 16 || (n > 0 && (!pos || !taylor || !acc))) return ORACLE_EINVAL;
    const int ncomp = (p + 1) * (p + 2) * (p + 3) / 6;
    const double s = (double)K / L;
    for (int64_t i = 0; i < n; i++) {
        double t[3];
        int c[3];
        for (int d = 0; d < 3; d++) {
            double xt;
            c[d] = axis_cell((double)pos[3 * i + d], L, s, K, &xt);
            t[d] = xt * s - ((double)c[d] + 0.5);
        }
        double pw3[3][17];
        for (int d = 0; d < 3; d++) {
            pw3[d][0] = 1.0;
            for (int q = 1; q <= p; q++) pw3[d][q] = pw3[d][q - 1] * t[d];
        }
        const double *T = taylor + (((int64_t)c[0] * K + c[1]) * K + c[2]) * ncomp;
        double gx = 0.0, gy = 0.0, gz = 0.0;
        int idx = 0;
        for (int deg = 0; deg <= p; deg++)
            for (int a = deg; a >= 0; a--)
                for (int b = deg - a; b >= 0; b--, idx++) {
                    const int k = deg - a - b;
                    if (a > 0) gx += T[idx] * a * pw3[0][a - 1] * pw3[1][b] * pw3[2][k];
                    if (b > 0) gy += T[idx] * b * pw3[0][a] * pw3[1][b - 1] * pw3[2][k];
                    if (k > 0) gz += T[idx] * k * pw3[0][a] * pw3[1][b] * pw3[2][k - 1];
                }
        acc[3 * i + 0] -= s * gx;
        acc[3 * i + 1] -= s * gy;
        acc[3 * i + 2] -= s * gz;
    }
    return ORACLE_OK;
}
