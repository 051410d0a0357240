/*
 * oracle.c -- plain, slow FP64 CPU oracle for the articulated-NeRF
 * deform-and-query path (InstantAvatar, arXiv 2212.10550).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header, table or constant with
 * the HIP library.
 *
 * Every function follows the passage of the paper it cites, in the paper's
 * order and notation, with scalar loops in double precision.  Where the
 * paper is silent the reading used is stated next to the code.  OpenMP only
 * parallelises the outer loop over independent samples or rays.
 *
 * Arrays are row-major C arrays of double unless stated:
 *   points      [n][3]
 *   bones B     [nb][3][4]   (rigid transform, canonical -> posed)
 *   skin grid W [Dz][Dy][Dx][nb]
 *   hash table  [L][T][F]
 *   MLP params  per layer: W [out][in], b [out]
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXB 64

/* Number of threads the parallel loops use (1 without OpenMP). */
int32_t oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of the parallel loops (timing only; results do not depend
 * on it: every parallel loop writes disjoint outputs). */
void oracle_set_num_threads(int32_t n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------ */
/* Sec. 3.2 (ray r = o + t d, N samples between near and far) and      */
/* Sec. 3.3 (samples in empty occupancy cells are skipped).            */
/*                                                                    */
/* The keep/skip decision is an integer decided by floating point, so  */
/* it is taken in the kernel's precision, FP32, with every operation   */
/* an individually rounded IEEE single operation (no contraction).     */
/* Readings: the occupancy grid lives in the normalised posed space and */
/* is applied before deformation; samples sit at the midpoints         */
/* t_k = t_near + (k + 1/2) dt of a uniform step; delta of every kept  */
/* sample is the uniform step dt (skipping equals sigma = 0).          */
/* ------------------------------------------------------------------ */
static int march_ray(const float o[3], const float d[3], const float lo[3], const float hi[3],
                     float *t_near_out, float *t_far_out)
{
    float tmin = -INFINITY, tmax = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (d[a] != 0.0f) {
            float ta = (lo[a] - o[a]) / d[a];
            float tb = (hi[a] - o[a]) / d[a];
            float t0 = ta < tb ? ta : tb;
            float t1 = ta < tb ? tb : ta;
            if (t0 > tmin) tmin = t0;
            if (t1 < tmax) tmax = t1;
        } else if (o[a] < lo[a] || o[a] > hi[a]) {
            return 0;
        }
    }
    float tn = tmin > 0.0f ? tmin : 0.0f;
    if (!(tmax > tn)) return 0;
    *t_near_out = tn;
    *t_far_out = tmax;
    return 1;
}

/* occ: uint8 [G][G][G] indexed [z][y][x], or NULL for "everything occupied".
 * Returns the total number of kept samples (which may exceed cap; then only
 * the first cap samples are written). */
int64_t oracle_march(const float *rays_o, const float *rays_d, int64_t R,
                     const uint8_t *occ, int32_t G, const float aabb[6],
                     float dt_fixed, int32_t n_per_ray, int32_t max_steps,
                     double *xs, double *ts, int64_t *ray_id, int64_t cap,
                     int64_t *ray_off, int32_t *ray_cnt, double *ray_dt)
{
    const float lo[3] = {aabb[0], aabb[1], aabb[2]};
    const float hi[3] = {aabb[3], aabb[4], aabb[5]};
    int64_t total = 0;
    for (int64_t r = 0; r < R; ++r) {
        const float *o = rays_o + 3 * r, *d = rays_d + 3 * r;
        float tn, tf, dt = 0.0f;
        int32_t cnt = 0;
        ray_off[r] = total;
        if (march_ray(o, d, lo, hi, &tn, &tf)) {
            dt = n_per_ray > 0 ? (tf - tn) / (float)n_per_ray : dt_fixed;
            for (int32_t k = 0; k < max_steps; ++k) {
                float t = tn + ((float)k + 0.5f) * dt;
                if (!(t < tf)) break;
                float x[3];
                int keep = 1;
                int cell[3];
                for (int a = 0; a < 3; ++a) {
                    x[a] = o[a] + t * d[a];
                    float u = (x[a] - lo[a]) / (hi[a] - lo[a]) * (float)G;
                    int c = (int)floorf(u);
                    cell[a] = c < 0 ? 0 : (c > G - 1 ? G - 1 : c);
                }
                if (occ) keep = occ[((int64_t)cell[2] * G + cell[1]) * G + cell[0]] != 0;
                if (!keep) continue;
                if (total < cap) {
                    for (int a = 0; a < 3; ++a) xs[3 * total + a] = (double)x[a];
                    ts[total] = (double)t;
                    ray_id[total] = r;
                }
                ++total;
                ++cnt;
            }
        }
        ray_cnt[r] = cnt;
        ray_dt[r] = (double)dt;
    }
    ray_off[R] = total;
    return total;
}

/* ------------------------------------------------------------------ */
/* Sec. 3.1, Eq. (5)-(6): skinning weights w(x) from a low-resolution   */
/* voxel grid.  Reading: trilinear interpolation with vertices on the  */
/* box corners (align-corners) and coordinates clamped to the box, so  */
/* the weights are constant (zero gradient) outside it along a clamped */
/* axis.  Also returns dw_b/dx (analytic gradient of the interpolant;  */
/* on a cell face the cell chosen by floor is used).                    */
/* ------------------------------------------------------------------ */
typedef struct {
    const double *W;
    int dx, dy, dz, nb;
    double lo[3], hi[3];
} skin_t;

static void skin_eval(const skin_t *s, const double x[3], double *w, double (*dw)[3])
{
    const int D[3] = {s->dx, s->dy, s->dz};
    int i0[3];
    double f[3], scale[3];
    for (int a = 0; a < 3; ++a) {
        double p = (x[a] - s->lo[a]) / (s->hi[a] - s->lo[a]) * (double)(D[a] - 1);
        scale[a] = (double)(D[a] - 1) / (s->hi[a] - s->lo[a]);
        if (p < 0.0) { p = 0.0; scale[a] = 0.0; }
        if (p > (double)(D[a] - 1)) { p = (double)(D[a] - 1); scale[a] = 0.0; }
        int i = (int)floor(p);
        if (i > D[a] - 2) i = D[a] - 2;
        if (i < 0) i = 0;
        i0[a] = i;
        f[a] = p - (double)i;
    }
    for (int b = 0; b < s->nb; ++b) {
        w[b] = 0.0;
        if (dw) dw[b][0] = dw[b][1] = dw[b][2] = 0.0;
    }
    for (int c = 0; c < 8; ++c) {
        const int cx = c & 1, cy = (c >> 1) & 1, cz = (c >> 2) & 1;
        const double wx = cx ? f[0] : 1.0 - f[0];
        const double wy = cy ? f[1] : 1.0 - f[1];
        const double wz = cz ? f[2] : 1.0 - f[2];
        const double sx = cx ? 1.0 : -1.0, sy = cy ? 1.0 : -1.0, sz = cz ? 1.0 : -1.0;
        const double *Wc = s->W + ((((int64_t)(i0[2] + cz) * s->dy + (i0[1] + cy)) * s->dx + (i0[0] + cx)) * s->nb);
        const double tri = wx * wy * wz;
        for (int b = 0; b < s->nb; ++b) {
            w[b] += tri * Wc[b];
            if (dw) {
                dw[b][0] += sx * wy * wz * scale[0] * Wc[b];
                dw[b][1] += wx * sy * wz * scale[1] * Wc[b];
                dw[b][2] += wx * wy * sz * scale[2] * Wc[b];
            }
        }
    }
}

/* Eq. (7): x' = sum_i w_i(x) B_i x  (x homogeneous). */
static void lbs_forward(const skin_t *s, const double *B, const double x[3], double y[3])
{
    double w[MAXB];
    skin_eval(s, x, w, NULL);
    y[0] = y[1] = y[2] = 0.0;
    for (int b = 0; b < s->nb; ++b) {
        const double *Bb = B + 12 * b;
        for (int i = 0; i < 3; ++i)
            y[i] += w[b] * (Bb[4 * i + 0] * x[0] + Bb[4 * i + 1] * x[1] + Bb[4 * i + 2] * x[2] + Bb[4 * i + 3]);
    }
}

/* Residual g(x) = LBS(x) - x' and (optionally) its Jacobian
 * J = sum_b w_b M_b + sum_b (B_b x_h) (grad w_b)^T, M_b the linear block. */
static void lbs_residual(const skin_t *s, const double *B, const double xp[3], const double x[3],
                         double g[3], double J[3][3])
{
    double w[MAXB], dw[MAXB][3];
    skin_eval(s, x, w, J ? dw : NULL);
    g[0] = -xp[0]; g[1] = -xp[1]; g[2] = -xp[2];
    if (J) memset(J, 0, sizeof(double) * 9);
    for (int b = 0; b < s->nb; ++b) {
        const double *Bb = B + 12 * b;
        for (int i = 0; i < 3; ++i) {
            const double yi = Bb[4 * i + 0] * x[0] + Bb[4 * i + 1] * x[1] + Bb[4 * i + 2] * x[2] + Bb[4 * i + 3];
            g[i] += w[b] * yi;
            if (J)
                for (int j = 0; j < 3; ++j) J[i][j] += w[b] * Bb[4 * i + j] + yi * dw[b][j];
        }
    }
}

static double det3(const double A[3][3])
{
    return A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1])
         - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0])
         + A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
}

/* Inverse by the adjugate; returns the determinant. */
static double inv3(const double A[3][3], double Ai[3][3])
{
    const double det = det3(A);
    const double id = 1.0 / det;
    Ai[0][0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) * id;
    Ai[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) * id;
    Ai[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) * id;
    Ai[1][0] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) * id;
    Ai[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) * id;
    Ai[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) * id;
    Ai[2][0] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) * id;
    Ai[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) * id;
    Ai[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) * id;
    return det;
}

/* Solve A x = b by Gaussian elimination with partial pivoting. */
static int solve3(const double Ain[3][3], const double bin[3], double x[3])
{
    double A[3][4];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) A[i][j] = Ain[i][j];
        A[i][3] = bin[i];
    }
    for (int c = 0; c < 3; ++c) {
        int p = c;
        for (int r = c + 1; r < 3; ++r)
            if (fabs(A[r][c]) > fabs(A[p][c])) p = r;
        if (A[p][c] == 0.0) return 0;
        if (p != c)
            for (int j = 0; j < 4; ++j) { double t = A[c][j]; A[c][j] = A[p][j]; A[p][j] = t; }
        for (int r = c + 1; r < 3; ++r) {
            const double m = A[r][c] / A[c][c];
            for (int j = c; j < 4; ++j) A[r][j] -= m * A[c][j];
        }
    }
    for (int i = 2; i >= 0; --i) {
        double v = A[i][3];
        for (int j = i + 1; j < 3; ++j) v -= A[i][j] * x[j];
        x[i] = v / A[i][i];
    }
    return 1;
}

static double norm3(const double v[3]) { return sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); }

static void make_skin(skin_t *s, const double *W, int dx, int dy, int dz, int nb, const double *skin_aabb)
{
    s->W = W; s->dx = dx; s->dy = dy; s->dz = dz; s->nb = nb;
    for (int a = 0; a < 3; ++a) { s->lo[a] = skin_aabb[a]; s->hi[a] = skin_aabb[3 + a]; }
}

/* Exported: skinning weights (and gradients) at n points, for tests. */
void oracle_skin_weights(const double *W, int32_t dx, int32_t dy, int32_t dz, int32_t nb, const double *skin_aabb,
                         const double *x, int64_t n, double *w, double *dw)
{
    skin_t s;
    make_skin(&s, W, dx, dy, dz, nb, skin_aabb);
    for (int64_t i = 0; i < n; ++i)
        skin_eval(&s, x + 3 * i, w + (int64_t)nb * i, dw ? (double (*)[3])(dw + (int64_t)3 * nb * i) : NULL);
}

/* Exported: forward LBS, Eq. (7), at n canonical points. */
void oracle_lbs(const double *B, int32_t nb, const double *W, int32_t dx, int32_t dy, int32_t dz,
                const double *skin_aabb, const double *x, int64_t n, double *xp)
{
    skin_t s;
    make_skin(&s, W, dx, dy, dz, nb, skin_aabb);
    for (int64_t i = 0; i < n; ++i) lbs_forward(&s, B, x + 3 * i, xp + 3 * i);
}

/* ------------------------------------------------------------------ */
/* Sec. 3.1: the canonical correspondence x* of a posed point x' is the */
/* root of Eq. (7), found by root finding as in Fast-SNARF.  Reading   */
/* (the paper defers the solver to Fast-SNARF): Broyden's method,      */
/* started once per bone at x0 = B_i^{-1} x' with H0 = J(x0)^{-1}, the */
/* "good" Broyden update in Sherman-Morrison form, at most max_iter    */
/* steps, stopping when ||g|| < tol_stop; an init is valid when its    */
/* final ||g|| < tol_valid and its point lies in the canonical box; the */
/* valid init with the lowest residual is kept (ties: lowest index).    */
/* The chosen root is then polished by Newton's method with the exact  */
/* Jacobian, and the set of distinct valid roots is reported.          */
/* ------------------------------------------------------------------ */
static int broyden_one(const skin_t *s, const double *B, const double xp[3], int init,
                       int max_iter, double tol_stop, double x_out[3], double *r_out, int *it_out)
{
    const double *Bi = B + 12 * init;
    double M[3][3], Mi[3][3], J[3][3], H[3][3], g[3], x[3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) M[i][j] = Bi[4 * i + j];
    const double dM = inv3(M, Mi);
    *it_out = 0;
    if (fabs(dM) < 1e-12) { *r_out = INFINITY; return 0; }
    for (int i = 0; i < 3; ++i)
        x[i] = Mi[i][0] * (xp[0] - Bi[3]) + Mi[i][1] * (xp[1] - Bi[7]) + Mi[i][2] * (xp[2] - Bi[11]);
    lbs_residual(s, B, xp, x, g, J);
    if (fabs(det3(J)) < 1e-12) { memcpy(x_out, x, sizeof x); *r_out = INFINITY; return 0; }
    inv3(J, H);
    int k = 0;
    for (; k < max_iter; ++k) {
        if (norm3(g) < tol_stop) break;
        double dx[3], xn[3], gn[3], dg[3], Hdg[3], dxH[3];
        for (int i = 0; i < 3; ++i) dx[i] = -(H[i][0] * g[0] + H[i][1] * g[1] + H[i][2] * g[2]);
        for (int i = 0; i < 3; ++i) xn[i] = x[i] + dx[i];
        lbs_residual(s, B, xp, xn, gn, NULL);
        for (int i = 0; i < 3; ++i) dg[i] = gn[i] - g[i];
        for (int i = 0; i < 3; ++i) Hdg[i] = H[i][0] * dg[0] + H[i][1] * dg[1] + H[i][2] * dg[2];
        for (int j = 0; j < 3; ++j) dxH[j] = dx[0] * H[0][j] + dx[1] * H[1][j] + dx[2] * H[2][j];
        const double den = dx[0] * Hdg[0] + dx[1] * Hdg[1] + dx[2] * Hdg[2];
        memcpy(x, xn, sizeof x);
        memcpy(g, gn, sizeof g);
        if (fabs(den) < 1e-30) { ++k; memcpy(x_out, x, sizeof x); *it_out = k; *r_out = INFINITY; return 0; }
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) H[i][j] += (dx[i] - Hdg[i]) * dxH[j] / den;
    }
    memcpy(x_out, x, sizeof x);
    *it_out = k;
    *r_out = norm3(g);
    return 1;
}

static void newton_polish(const skin_t *s, const double *B, const double xp[3], double x[3])
{
    double best[3], g[3], J[3][3], dx[3];
    memcpy(best, x, sizeof best);
    lbs_residual(s, B, xp, x, g, J);
    double rbest = norm3(g);
    for (int it = 0; it < 50 && rbest >= 1e-13; ++it) {
        if (!solve3(J, g, dx)) break;
        for (int i = 0; i < 3; ++i) x[i] -= dx[i];
        lbs_residual(s, B, xp, x, g, J);
        const double r = norm3(g);
        if (r < rbest) { rbest = r; memcpy(best, x, sizeof best); }
    }
    memcpy(x, best, sizeof best);
}

static int in_box(const double x[3], const double *box)
{
    for (int a = 0; a < 3; ++a)
        if (x[a] < box[a] || x[a] > box[3 + a]) return 0;
    return 1;
}

/* xp [S][3]; outputs: xc [S][3] (polished chosen root, or the unpolished
 * final iterate of init 0 when invalid), bone [S] (chosen init, -1 invalid),
 * resid [S] (chosen init's Broyden residual), and optionally per-init final
 * iterates init_x [S][nb][3], residuals init_r [S][nb], step counts init_it
 * [S][nb], and the distinct polished valid roots n_roots [S], roots [S][nb][3]. */
void oracle_deform(const double *xp, int64_t S, const double *B, int32_t nb,
                   const double *W, int32_t dx, int32_t dy, int32_t dz, const double *skin_aabb,
                   const double *hash_aabb, int32_t max_iter, double tol_stop, double tol_valid,
                   double *xc, int32_t *bone, double *resid,
                   double *init_x, double *init_r, int32_t *init_it, int32_t *n_roots, double *roots)
{
    skin_t s;
    make_skin(&s, W, dx, dy, dz, nb, skin_aabb);
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t n = 0; n < S; ++n) {
        const double *p = xp + 3 * n;
        double xi[MAXB][3], ri[MAXB];
        int iti[MAXB], ok[MAXB];
        for (int i = 0; i < nb; ++i) {
            ok[i] = broyden_one(&s, B, p, i, max_iter, tol_stop, xi[i], &ri[i], &iti[i]);
            ok[i] = ok[i] && ri[i] < tol_valid && in_box(xi[i], hash_aabb);
        }
        int best = -1;
        for (int i = 0; i < nb; ++i)
            if (ok[i] && (best < 0 || ri[i] < ri[best])) best = i;
        bone[n] = best;
        resid[n] = best >= 0 ? ri[best] : INFINITY;
        double x[3];
        memcpy(x, xi[best >= 0 ? best : 0], sizeof x);
        if (best >= 0) newton_polish(&s, B, p, x);
        memcpy(xc + 3 * n, x, sizeof x);
        if (init_x) memcpy(init_x + (int64_t)3 * nb * n, xi, sizeof(double) * 3 * nb);
        if (init_r) for (int i = 0; i < nb; ++i) init_r[(int64_t)nb * n + i] = ri[i];
        if (init_it) for (int i = 0; i < nb; ++i) init_it[(int64_t)nb * n + i] = iti[i];
        if (n_roots) {
            int cnt = 0;
            double *rts = roots + (int64_t)3 * nb * n;
            for (int i = 0; i < nb; ++i) {
                if (!ok[i]) continue;
                double y[3];
                memcpy(y, xi[i], sizeof y);
                newton_polish(&s, B, p, y);
                int dup = 0;
                for (int c = 0; c < cnt; ++c) {
                    const double e[3] = {rts[3 * c] - y[0], rts[3 * c + 1] - y[1], rts[3 * c + 2] - y[2]};
                    if (norm3(e) < 1e-6) dup = 1;
                }
                if (!dup) { memcpy(rts + 3 * cnt, y, sizeof y); ++cnt; }
            }
            n_roots[n] = cnt;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Backward through the root finder by the implicit function theorem.  */
/* At a root, g(x*, x', B, W) = 0, so dx* = -J^{-1} dg; with u = dL/dx* */
/* and v = J^{-T} u:  dL/dx' = v,  dL/dB_b = -w_b(x*) v x*_h^T,        */
/* dL/dW[c][b] = -tri_c(x*) v^T (B_b x*_h).  Invalid samples get zero.  */
/* Gradients are accumulated (+=) into grad_B and grad_W.              */
/* ------------------------------------------------------------------ */
void oracle_deform_bwd(const double *grad_xc, const double *xc, const int32_t *bone, int64_t S,
                       const double *B, int32_t nb, const double *W, int32_t dx, int32_t dy, int32_t dz,
                       const double *skin_aabb, double *grad_xp, double *grad_B, double *grad_W)
{
    skin_t s;
    make_skin(&s, W, dx, dy, dz, nb, skin_aabb);
    const int D[3] = {dx, dy, dz};
    for (int64_t n = 0; n < S; ++n) {
        double *gxp = grad_xp + 3 * n;
        gxp[0] = gxp[1] = gxp[2] = 0.0;
        if (bone[n] < 0) continue;
        const double *x = xc + 3 * n;
        double g[3], J[3][3], JT[3][3], v[3];
        const double zero[3] = {0, 0, 0};
        lbs_residual(&s, B, zero, x, g, J);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) JT[i][j] = J[j][i];
        if (!solve3(JT, grad_xc + 3 * n, v)) continue;
        memcpy(gxp, v, sizeof v);
        double w[MAXB];
        skin_eval(&s, x, w, NULL);
        const double xh[4] = {x[0], x[1], x[2], 1.0};
        for (int b = 0; b < nb; ++b)
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 4; ++j) grad_B[12 * b + 4 * i + j] -= w[b] * v[i] * xh[j];
        /* trilinear corner weights at x* (same cell rule as skin_eval) */
        int i0[3];
        double f[3];
        for (int a = 0; a < 3; ++a) {
            double p = (x[a] - s.lo[a]) / (s.hi[a] - s.lo[a]) * (double)(D[a] - 1);
            if (p < 0.0) p = 0.0;
            if (p > (double)(D[a] - 1)) p = (double)(D[a] - 1);
            int i = (int)floor(p);
            if (i > D[a] - 2) i = D[a] - 2;
            if (i < 0) i = 0;
            i0[a] = i;
            f[a] = p - (double)i;
        }
        for (int c = 0; c < 8; ++c) {
            const int cx = c & 1, cy = (c >> 1) & 1, cz = (c >> 2) & 1;
            const double tri = (cx ? f[0] : 1 - f[0]) * (cy ? f[1] : 1 - f[1]) * (cz ? f[2] : 1 - f[2]);
            double *gW = grad_W + ((((int64_t)(i0[2] + cz) * dy + (i0[1] + cy)) * dx + (i0[0] + cx)) * nb);
            for (int b = 0; b < nb; ++b) {
                const double *Bb = B + 12 * b;
                double vy = 0.0;
                for (int i = 0; i < 3; ++i)
                    vy += v[i] * (Bb[4 * i] * xh[0] + Bb[4 * i + 1] * xh[1] + Bb[4 * i + 2] * xh[2] + Bb[4 * i + 3]);
                gW[b] -= tri * vy;
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* Sec. 3.1 (Instant-NGP): multiresolution hash encoding.  The paper   */
/* only names it; the level rule follows Instant-NGP's definition:     */
/* N_l = floor(N_min * b^l); vertices at integer multiples of 1/N_l of  */
/* the canonical box; a level is stored densely when (N_l+1)^3 <= T,    */
/* otherwise vertex v maps to (v_x*1 xor v_y*2654435761 xor             */
/* v_z*805459861) mod 2^32 mod T.  Features of the eight surrounding    */
/* vertices are trilinearly interpolated and the levels concatenated.  */
/* Points are clamped to the box first.                                */
/* ------------------------------------------------------------------ */
void oracle_hash_resolutions(int32_t L, double base, double growth, int32_t *res)
{
    for (int l = 0; l < L; ++l) res[l] = (int32_t)floor(base * pow(growth, (double)l));
}

static uint64_t hash_index(int64_t T, int32_t N, const int64_t v[3])
{
    const uint64_t side = (uint64_t)N + 1;
    if (side * side * side <= (uint64_t)T)
        return (uint64_t)v[0] + side * ((uint64_t)v[1] + side * (uint64_t)v[2]);
    const uint32_t h = (uint32_t)((uint32_t)v[0] * 1u) ^ (uint32_t)((uint32_t)v[1] * 2654435761u)
                     ^ (uint32_t)((uint32_t)v[2] * 805459861u);
    return (uint64_t)h % (uint64_t)T;
}

typedef struct {
    int64_t idx[8];
    double w[8];
    double dw[8][3]; /* d w_c / d x (in canonical units) */
} cell_t;

static void hash_cell(int32_t N, int64_t T, const double lo[3], const double hi[3], const double x[3], cell_t *c)
{
    int64_t v0[3];
    double f[3], sc[3];
    for (int a = 0; a < 3; ++a) {
        double xn = (x[a] - lo[a]) / (hi[a] - lo[a]);
        sc[a] = (double)N / (hi[a] - lo[a]);
        if (xn < 0.0) { xn = 0.0; sc[a] = 0.0; }
        if (xn > 1.0) { xn = 1.0; sc[a] = 0.0; }
        const double u = xn * (double)N;
        int64_t i = (int64_t)floor(u);
        if (i > N - 1) i = N - 1;
        if (i < 0) i = 0;
        v0[a] = i;
        f[a] = u - (double)i;
    }
    for (int k = 0; k < 8; ++k) {
        const int cx = k & 1, cy = (k >> 1) & 1, cz = (k >> 2) & 1;
        const int64_t v[3] = {v0[0] + cx, v0[1] + cy, v0[2] + cz};
        const double wx = cx ? f[0] : 1 - f[0], wy = cy ? f[1] : 1 - f[1], wz = cz ? f[2] : 1 - f[2];
        c->idx[k] = (int64_t)hash_index(T, N, v);
        c->w[k] = wx * wy * wz;
        c->dw[k][0] = (cx ? 1.0 : -1.0) * wy * wz * sc[0];
        c->dw[k][1] = wx * (cy ? 1.0 : -1.0) * wz * sc[1];
        c->dw[k][2] = wx * wy * (cz ? 1.0 : -1.0) * sc[2];
    }
}

/* x [S][3]; valid [S] (nullable; invalid samples get zero features);
 * table [L][T][F]; feat [S][L*F]. */
void oracle_hash_encode(const double *x, const int32_t *valid, int64_t S, const double *table,
                        int32_t L, int32_t F, int64_t T, const int32_t *res, const double *aabb, double *feat)
{
    #pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < S; ++n) {
        double *out = feat + (int64_t)n * L * F;
        for (int k = 0; k < L * F; ++k) out[k] = 0.0;
        if (valid && valid[n] < 0) continue;
        for (int l = 0; l < L; ++l) {
            cell_t c;
            hash_cell(res[l], T, aabb, aabb + 3, x + 3 * n, &c);
            for (int k = 0; k < 8; ++k)
                for (int f = 0; f < F; ++f)
                    out[l * F + f] += c.w[k] * table[((int64_t)l * T + c.idx[k]) * F + f];
        }
    }
}

/* Backward: grad_table[l, idx_c, :] += w_c * dL/dfeat_l  (accumulated);
 * grad_x [S][3] (nullable, overwritten) = sum_l sum_c (grad w_c) (theta_c . dL/dfeat_l). */
void oracle_hash_encode_bwd(const double *grad_feat, const double *x, const int32_t *valid, int64_t S,
                            const double *table, int32_t L, int32_t F, int64_t T, const int32_t *res,
                            const double *aabb, double *grad_table, double *grad_x)
{
    for (int64_t n = 0; n < S; ++n) {
        double gx[3] = {0, 0, 0};
        if (!(valid && valid[n] < 0)) {
            const double *gf = grad_feat + (int64_t)n * L * F;
            for (int l = 0; l < L; ++l) {
                cell_t c;
                hash_cell(res[l], T, aabb, aabb + 3, x + 3 * n, &c);
                for (int k = 0; k < 8; ++k) {
                    double dot = 0.0;
                    for (int f = 0; f < F; ++f) {
                        grad_table[((int64_t)l * T + c.idx[k]) * F + f] += c.w[k] * gf[l * F + f];
                        dot += table[((int64_t)l * T + c.idx[k]) * F + f] * gf[l * F + f];
                    }
                    for (int a = 0; a < 3; ++a) gx[a] += c.dw[k][a] * dot;
                }
            }
        }
        if (grad_x) for (int a = 0; a < 3; ++a) grad_x[3 * n + a] = gx[a];
    }
}

/* ------------------------------------------------------------------ */
/* Sec. 3.1, Eq. (1)-(2): the shallow MLP decoding the concatenated     */
/* features into density and colour.  Reading: ReLU hidden layers, a    */
/* linear output layer, sigma = exp(o_0) (positive, log-space density  */
/* as in Instant-NGP) and c = sigmoid(o_1..3).  Invalid samples give    */
/* sigma = 0, c = 0.                                                    */
/* ------------------------------------------------------------------ */
#define MAXW 256

static void mlp_layer_offsets(const int32_t *widths, int32_t n_layers, int64_t *offW, int64_t *offb)
{
    int64_t o = 0;
    for (int l = 0; l < n_layers; ++l) {
        offW[l] = o;
        o += (int64_t)widths[l] * widths[l + 1];
        offb[l] = o;
        o += widths[l + 1];
    }
}

/* BF16 storage (the reduced-precision form; the paper fixes no precision,
 * so a decision taken on a stored value -- a ReLU mask -- is taken on the
 * value the kernels store, in their precision): x is rounded to IEEE single,
 * then to the nearest bfloat16 (8 significant bits), ties to even. */
static double round_bf16(double x)
{
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, sizeof u);
    if ((u & 0x7f800000u) != 0x7f800000u) {   /* finite: round the low 16 bits away */
        u += 0x7fffu + ((u >> 16) & 1u);
        u &= 0xffff0000u;
    } else if (u & 0x007fffffu) {
        u |= 0x00400000u;                      /* NaN stays NaN */
        u &= 0xffff0000u;
    }
    memcpy(&f, &u, sizeof f);
    return (double)f;
}

static double store_act(double x, int32_t bf16) { return bf16 ? round_bf16(x) : x; }

/* bf16 != 0: the BF16 storage form.  The input features and every stored
 * activation are bfloat16 (the features are rounded on input, each hidden
 * activation after its ReLU), and every weight matrix is used rounded to
 * bfloat16; biases stay as given and the sums are exact (FP64).  With
 * bf16 == 0 every value is FP64. */
void oracle_mlp_fwd(const double *feat, const int32_t *valid, int64_t S, const double *params,
                    const int32_t *widths, int32_t n_layers, int32_t bf16, double *sigma, double *rgb)
{
    int64_t offW[16], offb[16];
    mlp_layer_offsets(widths, n_layers, offW, offb);
    #pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < S; ++n) {
        double a[MAXW], h[MAXW];
        if (valid && valid[n] < 0) {
            sigma[n] = 0.0;
            rgb[3 * n] = rgb[3 * n + 1] = rgb[3 * n + 2] = 0.0;
            continue;
        }
        for (int i = 0; i < widths[0]; ++i) a[i] = store_act(feat[n * widths[0] + i], bf16);
        for (int l = 0; l < n_layers; ++l) {
            const double *Wl = params + offW[l], *bl = params + offb[l];
            for (int o = 0; o < widths[l + 1]; ++o) {
                double z = bl[o];
                for (int i = 0; i < widths[l]; ++i) z += store_act(Wl[(int64_t)o * widths[l] + i], bf16) * a[i];
                h[o] = l < n_layers - 1 ? store_act(z < 0.0 ? 0.0 : z, bf16) : z;
            }
            memcpy(a, h, sizeof(double) * widths[l + 1]);
        }
        sigma[n] = exp(a[0]);
        for (int k = 0; k < 3; ++k) rgb[3 * n + k] = 1.0 / (1.0 + exp(-a[1 + k]));
    }
}

/* grad_params accumulated (+=); grad_feat [S][widths[0]] overwritten.
 * bf16 != 0: the BF16 storage form of the forward above; each layer's
 * backpropagated delta, after its ReLU mask (taken on the pre-activation),
 * is stored as bfloat16 where it multiplies (the weight-gradient products
 * and the product with the layer's rounded weights), while the bias
 * gradients sum the deltas unrounded. */
void oracle_mlp_bwd(const double *grad_sigma, const double *grad_rgb, const double *feat, const int32_t *valid,
                    int64_t S, const double *params, const int32_t *widths, int32_t n_layers, int32_t bf16,
                    double *grad_params, double *grad_feat)
{
    int64_t offW[16], offb[16];
    mlp_layer_offsets(widths, n_layers, offW, offb);
    for (int64_t n = 0; n < S; ++n) {
        double act[17][MAXW], pre[16][MAXW], d[MAXW], dn[MAXW], dq[MAXW];
        double *gfeat = grad_feat + n * widths[0];
        for (int i = 0; i < widths[0]; ++i) gfeat[i] = 0.0;
        if (valid && valid[n] < 0) continue;
        for (int i = 0; i < widths[0]; ++i) act[0][i] = store_act(feat[n * widths[0] + i], bf16);
        for (int l = 0; l < n_layers; ++l) {
            const double *Wl = params + offW[l], *bl = params + offb[l];
            for (int o = 0; o < widths[l + 1]; ++o) {
                double z = bl[o];
                for (int i = 0; i < widths[l]; ++i) z += store_act(Wl[(int64_t)o * widths[l] + i], bf16) * act[l][i];
                pre[l][o] = z;
                act[l + 1][o] = l < n_layers - 1 ? store_act(z < 0.0 ? 0.0 : z, bf16) : z;
            }
        }
        const double *o = act[n_layers];
        const double sg = exp(o[0]);
        d[0] = grad_sigma[n] * sg;
        for (int k = 0; k < 3; ++k) {
            const double c = 1.0 / (1.0 + exp(-o[1 + k]));
            d[1 + k] = grad_rgb[3 * n + k] * c * (1.0 - c);
        }
        for (int k = 4; k < widths[n_layers]; ++k) d[k] = 0.0;
        for (int l = n_layers - 1; l >= 0; --l) {
            const double *Wl = params + offW[l];
            double *gW = grad_params + offW[l], *gb = grad_params + offb[l];
            if (l < n_layers - 1)
                for (int q = 0; q < widths[l + 1]; ++q)
                    if (pre[l][q] < 0.0) d[q] = 0.0;
            for (int q = 0; q < widths[l + 1]; ++q) {
                gb[q] += d[q];
                dq[q] = store_act(d[q], bf16);
                for (int i = 0; i < widths[l]; ++i) gW[(int64_t)q * widths[l] + i] += dq[q] * act[l][i];
            }
            for (int i = 0; i < widths[l]; ++i) {
                double v = 0.0;
                for (int q = 0; q < widths[l + 1]; ++q) v += store_act(Wl[(int64_t)q * widths[l] + i], bf16) * dq[q];
                dn[i] = v;
            }
            memcpy(d, dn, sizeof(double) * widths[l]);
        }
        for (int i = 0; i < widths[0]; ++i) gfeat[i] = d[i];
    }
}

/* ------------------------------------------------------------------ */
/* Sec. 3.2, Eq. (8): C = sum_i alpha_i prod_{j<i}(1 - alpha_j) c_i.   */
/* Readings: alpha_i = 1 - exp(-sigma_i delta_i) (the printed sign is a */
/* typo: it would give alpha < 0); delta_i is the uniform step of the  */
/* ray for every sample, the last included; the opacity                */
/* A = sum_i T_i alpha_i is returned beside C (no background); rays    */
/* terminate early (Sec. 3.4): sample i and all later ones are skipped */
/* iff T_i < T_thresh (T_thresh = 0 disables it).                      */
/* ------------------------------------------------------------------ */
void oracle_composite_fwd(const double *sigma, const double *rgb, const int64_t *ray_off, const double *ray_dt,
                          int64_t R, double T_thresh, double *color, double *opacity, int32_t *n_used,
                          double *T_final)
{
    #pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < R; ++r) {
        double T = 1.0, C[3] = {0, 0, 0}, A = 0.0;
        int32_t used = 0;
        for (int64_t i = ray_off[r]; i < ray_off[r + 1]; ++i) {
            if (T < T_thresh) break;
            const double alpha = 1.0 - exp(-sigma[i] * ray_dt[r]);
            const double w = T * alpha;
            for (int k = 0; k < 3; ++k) C[k] += w * rgb[3 * i + k];
            A += w;
            T *= 1.0 - alpha;
            ++used;
        }
        for (int k = 0; k < 3; ++k) color[3 * r + k] = C[k];
        opacity[r] = A;
        n_used[r] = used;
        T_final[r] = T;
    }
}

/* dL/dc_i = T_i alpha_i g_C;
 * dL/dsigma_i = delta_i [ T_{i+1} (g_C . c_i) - g_C . (sum_{j>i} T_j alpha_j c_j) ]
 *             + g_A delta_i T_final            (T_final = T after the last used sample).
 * Unused samples get zero. */
void oracle_composite_bwd(const double *grad_color, const double *grad_opacity, const double *sigma,
                          const double *rgb, const int64_t *ray_off, const double *ray_dt, const int32_t *n_used,
                          int64_t R, double *grad_sigma, double *grad_rgb)
{
    for (int64_t r = 0; r < R; ++r) {
        const int64_t b = ray_off[r], e = ray_off[r + 1], u = b + n_used[r];
        const double dt = ray_dt[r];
        const double *gC = grad_color + 3 * r;
        const double gA = grad_opacity ? grad_opacity[r] : 0.0;
        double Tfin = 1.0;
        for (int64_t i = b; i < u; ++i) Tfin *= exp(-sigma[i] * dt);
        for (int64_t i = b; i < e; ++i) {
            grad_sigma[i] = 0.0;
            grad_rgb[3 * i] = grad_rgb[3 * i + 1] = grad_rgb[3 * i + 2] = 0.0;
        }
        double T = 1.0;
        for (int64_t i = b; i < u; ++i) {
            const double alpha = 1.0 - exp(-sigma[i] * dt);
            const double w = T * alpha;
            const double Tn = T * (1.0 - alpha);
            double after[3] = {0, 0, 0}, Tj = Tn;
            for (int64_t j = i + 1; j < u; ++j) {
                const double aj = 1.0 - exp(-sigma[j] * dt);
                for (int k = 0; k < 3; ++k) after[k] += Tj * aj * rgb[3 * j + k];
                Tj *= 1.0 - aj;
            }
            double gc = 0.0, ga = 0.0;
            for (int k = 0; k < 3; ++k) {
                gc += gC[k] * rgb[3 * i + k];
                ga += gC[k] * after[k];
                grad_rgb[3 * i + k] = w * gC[k];
            }
            grad_sigma[i] = dt * (Tn * gc - ga) + gA * dt * Tfin;
            T = Tn;
        }
    }
}

/* Photometric L2 loss (the measurement's stand-in for the Huber loss of
 * Eq. (9)): L = mean over R*3 of (C - C_gt)^2; grad = dL/dC. */
double oracle_l2_loss(const double *color, const double *target, int64_t R, double *grad)
{
    double L = 0.0;
    const double inv = 1.0 / (3.0 * (double)R);
    for (int64_t i = 0; i < 3 * R; ++i) {
        const double e = color[i] - target[i];
        L += e * e * inv;
        if (grad) grad[i] = 2.0 * e * inv;
    }
    return L;
}

/* ------------------------------------------------------------------ */
/* Learned root initialiser (an addition to the method; not in the paper).  */
/* An MLP maps (x', pose) -> (bone logits, canonical offset):          */
/* input = (x'_xyz, then per bone axis-angle(3) and translation(3)),   */
/* ReLU hidden layers, linear outputs: nb logits then 3 offsets.       */
/* The predicted start is x0 = B_k^{-1} x' + offset with k = argmax     */
/* of the logits (ties: lowest bone).                                  */
/* params: per layer W [out][in] row-major, then b [out].              */
/* ------------------------------------------------------------------ */
void oracle_rootinit_fwd(const double *xp, int64_t S, const double *pose, int32_t nb, const double *params,
                         int32_t hidden, const double *B, int32_t *bone, double *x0)
{
    const int nin = 3 + 6 * nb, nout = nb + 3;
    const int widths[4] = {nin, hidden, hidden, nout};
    #pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < S; ++n) {
        double a[MAXW], h[MAXW];
        for (int i = 0; i < 3; ++i) a[i] = xp[3 * n + i];
        for (int i = 0; i < 6 * nb; ++i) a[3 + i] = pose[i];
        int64_t off = 0;
        for (int l = 0; l < 3; ++l) {
            const double *Wl = params + off;
            const double *bl = Wl + (int64_t)widths[l] * widths[l + 1];
            for (int o = 0; o < widths[l + 1]; ++o) {
                double z = bl[o];
                for (int i = 0; i < widths[l]; ++i) z += Wl[(int64_t)o * widths[l] + i] * a[i];
                h[o] = (l < 2 && z < 0.0) ? 0.0 : z;
            }
            memcpy(a, h, sizeof(double) * widths[l + 1]);
            off += (int64_t)widths[l] * widths[l + 1] + widths[l + 1];
        }
        int k = 0;
        for (int b = 1; b < nb; ++b)
            if (a[b] > a[k]) k = b;
        bone[n] = k;
        const double *Bk = B + 12 * k;
        double M[3][3], Mi[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) M[i][j] = Bk[4 * i + j];
        inv3(M, Mi);
        for (int i = 0; i < 3; ++i)
            x0[3 * n + i] = Mi[i][0] * (xp[3 * n] - Bk[3]) + Mi[i][1] * (xp[3 * n + 1] - Bk[7])
                          + Mi[i][2] * (xp[3 * n + 2] - Bk[11]) + a[nb + i];
    }
}

/* Guided root finding: one Broyden solve from the given start x0 (same
 * iteration as oracle_deform's per-bone solves); it is accepted when its
 * residual is below tol_valid and its point lies in the canonical box.
 * Otherwise the sample falls back to the multi-init solve of oracle_deform.
 * Outputs: xc (polished), bone (the guide's bone on success, the chosen
 * init on fallback, -1 invalid), steps [S] (guided steps plus, on fallback,
 * every init's steps), fallback [S] (0/1). */
void oracle_deform_guided(const double *xp, int64_t S, const double *x0, const int32_t *guide_bone,
                          const double *B, int32_t nb, const double *W, int32_t dx, int32_t dy, int32_t dz,
                          const double *skin_aabb, const double *hash_aabb, int32_t max_iter, double tol_stop,
                          double tol_valid, double *xc, int32_t *bone, int32_t *steps, int32_t *fallback)
{
    skin_t s;
    make_skin(&s, W, dx, dy, dz, nb, skin_aabb);
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t n = 0; n < S; ++n) {
        const double *p = xp + 3 * n;
        double x[3], g[3], J[3][3], H[3][3], r = INFINITY;
        int k = 0, ok = 1;
        memcpy(x, x0 + 3 * n, sizeof x);
        lbs_residual(&s, B, p, x, g, J);
        if (fabs(det3(J)) < 1e-12) ok = 0;
        else inv3(J, H);
        for (; ok && k < max_iter; ++k) {
            if (norm3(g) < tol_stop) break;
            double dxv[3], xn[3], gn[3], dg[3], Hdg[3], dxH[3];
            for (int i = 0; i < 3; ++i) dxv[i] = -(H[i][0] * g[0] + H[i][1] * g[1] + H[i][2] * g[2]);
            for (int i = 0; i < 3; ++i) xn[i] = x[i] + dxv[i];
            lbs_residual(&s, B, p, xn, gn, NULL);
            for (int i = 0; i < 3; ++i) dg[i] = gn[i] - g[i];
            for (int i = 0; i < 3; ++i) Hdg[i] = H[i][0] * dg[0] + H[i][1] * dg[1] + H[i][2] * dg[2];
            for (int j = 0; j < 3; ++j) dxH[j] = dxv[0] * H[0][j] + dxv[1] * H[1][j] + dxv[2] * H[2][j];
            const double den = dxv[0] * Hdg[0] + dxv[1] * Hdg[1] + dxv[2] * Hdg[2];
            memcpy(x, xn, sizeof x);
            memcpy(g, gn, sizeof g);
            if (fabs(den) < 1e-30) { ok = 0; ++k; break; }
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) H[i][j] += (dxv[i] - Hdg[i]) * dxH[j] / den;
        }
        if (ok) r = norm3(g);
        steps[n] = k;
        if (ok && r < tol_valid && in_box(x, hash_aabb)) {
            newton_polish(&s, B, p, x);
            memcpy(xc + 3 * n, x, sizeof x);
            bone[n] = guide_bone[n];
            fallback[n] = 0;
            continue;
        }
        fallback[n] = 1;
        double xi[MAXB][3], ri[MAXB];
        int iti[MAXB], oki[MAXB], best = -1;
        for (int i = 0; i < nb; ++i) {
            oki[i] = broyden_one(&s, B, p, i, max_iter, tol_stop, xi[i], &ri[i], &iti[i]);
            oki[i] = oki[i] && ri[i] < tol_valid && in_box(xi[i], hash_aabb);
            steps[n] += iti[i];
            if (oki[i] && (best < 0 || ri[i] < ri[best])) best = i;
        }
        bone[n] = best;
        memcpy(x, xi[best >= 0 ? best : 0], sizeof x);
        if (best >= 0) newton_polish(&s, B, p, x);
        memcpy(xc + 3 * n, x, sizeof x);
    }
}
