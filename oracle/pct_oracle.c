/*
 * Plain CPU oracle for point-cloud tomography (Yang et al., "Efficient Global
 * Navigational Planning in 3D Structures based on Point Cloud Tomography").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant generator with the HIP library; neither includes
 * or links the other.
 *
 * Everything is written as plain loops in the order the paper states it:
 *   - tomogram construction: Algorithm 1, construction part, literally
 *     (every point against every plane, O(points x slices)), in FP32, which
 *     is exact because only max/min and comparisons are involved;
 *   - traversability: Eqs. (1)-(5) per cell in FP64, then the inflation
 *     of Eq. (6) as a direct 2-D sliding-window weighted max in FP64;
 *   - simplification: the sequential slice test of Sec. III-C with the
 *     unique-grid conditions of Eqs. (8)-(9);
 *   - trajectory cost sampling and every adjoint, in FP64.
 *
 * Readings of points where the paper is silent or ambiguous are stated at
 * each function.  Build: gcc -O2 -fno-fast-math -ffp-contract=off [-fopenmp].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    float x0, y0, res;
    int32_t nx, ny;
    float slice_dz;
} o_grid;

typedef struct {
    float d_min, d_ref, theta_b, theta_s, theta_p, c_barrier, alpha_d, alpha_b, alpha_s, d_inf, d_sm;
    int32_t patch_radius;
} o_robot;

int o_omp_threads(void) {
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the number of threads of the parallel loops (for timing the oracle on
 * one core as well as on all); no effect on any result. */
void o_set_threads(int n) {
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Sec. III-A: rasterize.  The paper names the step but not the rule.
 * Reading: cell (i, j) of a grid with origin (x0, y0) and resolution r holds
 * the points with floor((x - x0) / r) = i and floor((y - y0) / r) = j, where
 * the subtraction and the division are single correctly rounded FP32
 * operations.  Points outside [0, nx) x [0, ny) are not part of the map. */
static int o_rasterize(float x, float y, const o_grid* g, int* ix, int* iy) {
    float qx = (x - g->x0) / g->res;
    float qy = (y - g->y0) / g->res;
    if (!(qx >= 0.0f && qx < (float)g->nx)) return 0;
    if (!(qy >= 0.0f && qy < (float)g->ny)) return 0;
    *ix = (int)floorf(qx);
    *iy = (int)floorf(qy);
    return 1;
}

static int o_point_ok(const float* p) {
    return isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2]);
}

/* Algorithm 1, first line: the lowest point height.  Reading: taken over the
 * points that belong to the map (finite and inside the grid); the highest
 * height is taken over the same set because the plane count depends on it.
 * Returns the number of such points. */
int64_t o_extent(const float* xyz, int64_t n, const o_grid* g, float* zmin, float* zmax) {
    float lo = INFINITY, hi = -INFINITY;
    int64_t used = 0;
    for (int64_t u = 0; u < n; ++u) {
        const float* p = xyz + 3 * u;
        int ix, iy;
        if (!o_point_ok(p) || !o_rasterize(p[0], p[1], g, &ix, &iy)) continue;
        float z = p[2] + 0.0f; /* -0 becomes +0 */
        if (z < lo) lo = z;
        if (z > hi) hi = z;
        ++used;
    }
    *zmin = lo;
    *zmax = hi;
    return used;
}

/* Sec. III-A: planes spaced d_s apart, the first one d_s above the lowest
 * point, as many as needed for the last one to lie above the highest point.
 * Plane k (k = 0 .. N-1) sits at z_min + (k + 1) d_s, evaluated as one FP32
 * multiply followed by one FP32 add.  Returns N, -1 if two consecutive
 * planes coincide in FP32, -2 if more than `cap` planes would be needed. */
int o_planes(float zmin, float zmax, float ds, int cap, float* h) {
    for (int k = 0; k < cap; ++k) {
        float step = (float)(k + 1) * ds;
        float hk = zmin + step;
        h[k] = hk;
        if (k > 0 && !(hk > h[k - 1])) return -1;
        if (hk > zmax) return k + 1;
    }
    return -2;
}

/* Algorithm 1, construction loop, literally: every point is compared with
 * every plane.  The lower group of plane k (z at or below the plane) sets the
 * ground elevation by max, the upper group (z above the plane) sets the
 * ceiling by min.  The printed algorithm swaps the two inequalities; the text
 * of Sec. III-A (lower group projected up to the ground layer, upper group
 * down to the ceiling) decides, and the equality case stays with the ground.
 * Empty cells are invalid: ground -inf, ceiling +inf, ids -1.  The ids record
 * which point gives each value; on equal heights the lowest index wins.
 * Layout of every [N][ny][nx] array: x fastest. */
void o_build(const float* xyz, int64_t n, const o_grid* g, const float* h, int N,
             float* eG, float* eC, int32_t* aG, int32_t* aC) {
    const int64_t plane = (int64_t)g->nx * g->ny;
    for (int64_t i = 0; i < plane * N; ++i) {
        eG[i] = -INFINITY;
        eC[i] = INFINITY;
        if (aG) aG[i] = -1;
        if (aC) aC[i] = -1;
    }
#pragma omp parallel for schedule(static)
    for (int k = 0; k < N; ++k) {
        for (int64_t u = 0; u < n; ++u) {
            const float* p = xyz + 3 * u;
            int ix, iy;
            if (!o_point_ok(p) || !o_rasterize(p[0], p[1], g, &ix, &iy)) continue;
            float z = p[2] + 0.0f;
            int64_t c = (int64_t)k * plane + (int64_t)iy * g->nx + ix;
            if (z <= h[k]) {
                if (z > eG[c]) { eG[c] = z; if (aG) aG[c] = (int32_t)u; }
            } else {
                if (z < eC[c]) { eC[c] = z; if (aC) aC[c] = (int32_t)u; }
            }
        }
    }
}

/* The same loop restricted to the cells of a window [wx0, wx0+wnx) x
 * [wy0, wy0+wny) of the grid (cells are still assigned with the full grid's
 * rasterisation).  Outputs are [N][wny][wnx].  Lets a map too large for the
 * full O(points x slices) loop be checked window by window. */
void o_build_window(const float* xyz, int64_t n, const o_grid* g, const float* h, int N,
                    int wx0, int wy0, int wnx, int wny,
                    float* eG, float* eC, int32_t* aG, int32_t* aC) {
    const int64_t plane = (int64_t)wnx * wny;
    for (int64_t i = 0; i < plane * N; ++i) {
        eG[i] = -INFINITY;
        eC[i] = INFINITY;
        if (aG) aG[i] = -1;
        if (aC) aC[i] = -1;
    }
#pragma omp parallel for schedule(static)
    for (int k = 0; k < N; ++k) {
        for (int64_t u = 0; u < n; ++u) {
            const float* p = xyz + 3 * u;
            int ix, iy;
            if (!o_point_ok(p) || !o_rasterize(p[0], p[1], g, &ix, &iy)) continue;
            if (ix < wx0 || iy < wy0 || ix >= wx0 + wnx || iy >= wy0 + wny) continue;
            float z = p[2] + 0.0f;
            int64_t c = (int64_t)k * plane + (int64_t)(iy - wy0) * wnx + (ix - wx0);
            if (z <= h[k]) {
                if (z > eG[c]) { eG[c] = z; if (aG) aG[c] = (int32_t)u; }
            } else {
                if (z < eC[c]) { eC[c] = z; if (aC) aC[c] = (int32_t)u; }
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Sec. III-B, traversability of one slice, in FP64. */

static double o_g(const float* eG, int nx, int ny, int x, int y) {
    if (x < 0 || y < 0 || x >= nx || y >= ny) return -INFINITY;
    return (double)eG[(int64_t)y * nx + x];
}

/* Eq. (2): central finite differences g^x = (e(x+1) - e(x-1)) / 2r and
 * likewise g^y; m^xy = max(|g^x|, |g^y|), m^grad = |g|.  Reading: a stencil
 * that needs a neighbour outside the grid or without ground has no slope
 * estimate and counts as infinitely steep (both magnitudes +inf). */
static void o_slope(const float* eG, int nx, int ny, double res, int x, int y,
                    double* gx, double* gy, double* mxy, double* mgrad) {
    double l = o_g(eG, nx, ny, x - 1, y), r = o_g(eG, nx, ny, x + 1, y);
    double d = o_g(eG, nx, ny, x, y - 1), u = o_g(eG, nx, ny, x, y + 1);
    if (!isfinite(l) || !isfinite(r) || !isfinite(d) || !isfinite(u)) {
        *gx = *gy = 0.0;
        *mxy = *mgrad = INFINITY;
        return;
    }
    *gx = (r - l) / (2.0 * res);
    *gy = (u - d) / (2.0 * res);
    *mxy = fmax(fabs(*gx), fabs(*gy));
    *mgrad = sqrt((*gx) * (*gx) + (*gy) * (*gy));
}

/* Eq. (4): the step test compares the share p_s of gentle neighbours with
 * theta_p.  Reading: the patch is the (2 r_p + 1)^2 square minus its centre
 * (r_p = 1 unless the robot says otherwise); neighbours outside the grid or
 * without ground are not gentle; the denominator is fixed.  p_s > theta_p is
 * decided in integers as count > floor(theta_p * patch) (FP64 product). */
static int o_patch_threshold(const o_robot* rb) {
    int np = (2 * rb->patch_radius + 1) * (2 * rb->patch_radius + 1) - 1;
    return (int)floor((double)rb->theta_p * (double)np);
}

typedef struct {
    double cI, cG, cinit, mxy, mgrad, gx, gy, dI;
    int gentle, count, branch; /* branch: 0 no ground, 1 barrier, 2 gentle, 3 step, 4 step-barrier */
} o_cell;

static int o_is_gentle(const float* eG, int nx, int ny, double res, const o_robot* rb, int x, int y) {
    if (!isfinite(o_g(eG, nx, ny, x, y))) return 0;
    double gx, gy, mxy, mg;
    o_slope(eG, nx, ny, res, x, y, &gx, &gy, &mxy, &mg);
    return mg < (double)rb->theta_s;
}

/* One cell of Eqs. (1)-(5).  Reading for invalid layers: no ground gives the
 * barrier cost c^B (nothing to stand on); no ceiling gives an infinite
 * interval and hence c^I = 0.  Case order of Eq. (3)/(4): barrier test first,
 * then the gentle test, then the step test. */
static o_cell o_eval_cell(const float* eG, const float* eC, int nx, int ny, double res,
                          const o_robot* rb, int x, int y) {
    o_cell o;
    memset(&o, 0, sizeof o);
    const double cB = rb->c_barrier;
    double G = o_g(eG, nx, ny, x, y);
    double C = (double)eC[(int64_t)y * nx + x];
    o_slope(eG, nx, ny, res, x, y, &o.gx, &o.gy, &o.mxy, &o.mgrad);
    o.gentle = isfinite(G) && o.mgrad < (double)rb->theta_s;
    if (!isfinite(G)) {
        o.cinit = cB;
        o.cI = cB;
        o.cG = cB;
        o.dI = NAN;
        o.branch = 0;
        return o;
    }
    /* Eq. (1) */
    o.dI = C - G;
    if (o.dI < (double)rb->d_min) o.cI = cB;
    else o.cI = fmax(0.0, (double)rb->alpha_d * ((double)rb->d_ref - o.dI));
    /* Eqs. (3)-(4) */
    int rp = rb->patch_radius;
    o.count = 0;
    for (int dy = -rp; dy <= rp; ++dy)
        for (int dx = -rp; dx <= rp; ++dx)
            if (dx || dy) o.count += o_is_gentle(eG, nx, ny, res, rb, x + dx, y + dy);
    if (o.mxy > (double)rb->theta_b) {
        o.cG = cB;
        o.branch = 1;
    } else if (o.mgrad < (double)rb->theta_s) {
        double t = o.mgrad / (double)rb->theta_s;
        o.cG = (double)rb->alpha_s * t * t;
        o.branch = 2;
    } else if (o.count > o_patch_threshold(rb)) {
        double t = o.mxy / (double)rb->theta_b;
        o.cG = (double)rb->alpha_b * t * t;
        o.branch = 3;
    } else {
        o.cG = cB;
        o.branch = 4;
    }
    /* Eq. (5) */
    o.cinit = fmin(cB, o.cI + o.cG);
    return o;
}

/* Per-cell layers of one slice; every output pointer may be NULL. */
void o_layers(const float* eG, const float* eC, int nx, int ny, double res, const o_robot* rb,
              double* cI, double* cG, double* cinit, double* mxy, double* mgrad,
              uint8_t* gentle, int32_t* branch) {
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            o_cell o = o_eval_cell(eG, eC, nx, ny, res, rb, x, y);
            int64_t i = (int64_t)y * nx + x;
            if (cI) cI[i] = o.cI;
            if (cG) cG[i] = o.cG;
            if (cinit) cinit[i] = o.cinit;
            if (mxy) mxy[i] = o.mxy;
            if (mgrad) mgrad[i] = o.mgrad;
            if (gentle) gentle[i] = (uint8_t)o.gentle;
            if (branch) branch[i] = o.branch;
        }
}

/* Eq. (6): K(m,n) = max(0, min(1 - (d_mn - d_inf) / (d_sm - r_g), 1)) with
 * d_mn = r_g sqrt(m^2 + n^2), in FP64 from the float parameters.
 * Reading: the parameters are decimal values stored as floats, so lattice
 * distances that equal d_inf or the outer edge in decimal land a few 1e-8
 * off; weights within 1e-6 of 1 are taken as 1 and within 1e-6 of 0 as 0.
 * K is written as a (2 rmax + 1)^2 array, row n + rmax, column m + rmax.
 * Returns the support radius R, -1 if d_sm <= r_g, -2 if the support does
 * not fit in rmax. */
int o_kernel(double res, double d_inf, double d_sm, int rmax, double* K) {
    if (!(d_sm > res)) return -1;
    int w = 2 * rmax + 1, R = 0;
    for (int n = -rmax; n <= rmax; ++n)
        for (int m = -rmax; m <= rmax; ++m) {
            double d = res * sqrt((double)(m * m + n * n));
            double k = 1.0 - (d - d_inf) / (d_sm - res);
            k = fmax(0.0, fmin(k, 1.0));
            if (k >= 1.0 - 1e-6) k = 1.0;
            if (k <= 1e-6) k = 0.0;
            K[(n + rmax) * w + (m + rmax)] = k;
            if (k > 0.0) {
                int a = abs(m) > abs(n) ? abs(m) : abs(n);
                if (a > R) R = a;
            }
        }
    if (R >= rmax) return -2;
    return R;
}

/* Sec. III-B, last paragraph: sliding window; each output cell takes the
 * maximum over the window of kernel weight times initial cost.  Window cells
 * outside the grid are skipped. */
void o_inflate(const double* cinit, int nx, int ny, const double* K, int rmax, int R, double* cT) {
    int w = 2 * rmax + 1;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            double best = -INFINITY;
            for (int n = -R; n <= R; ++n)
                for (int m = -R; m <= R; ++m) {
                    double k = K[(n + rmax) * w + (m + rmax)];
                    int qx = x + m, qy = y + n;
                    if (k <= 0.0 || qx < 0 || qy < 0 || qx >= nx || qy >= ny) continue;
                    double v = k * cinit[(int64_t)qy * nx + qx];
                    if (v > best) best = v;
                }
            cT[(int64_t)y * nx + x] = best;
        }
}

#define O_RMAX 24

/* Algorithm 1, evaluation lines: c^init per slice, then inflation, for all
 * N slices.  Returns R, or a negative kernel error. */
int o_eval(const float* eG, const float* eC, int N, int nx, int ny, double res,
           const o_robot* rb, double* cT) {
    double K[(2 * O_RMAX + 1) * (2 * O_RMAX + 1)];
    int R = o_kernel(res, rb->d_inf, rb->d_sm, O_RMAX, K);
    if (R < 0) return R;
    const int64_t plane = (int64_t)nx * ny;
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k < N; ++k) {
        double* ci = (double*)malloc(sizeof(double) * plane);
        o_layers(eG + k * plane, eC + k * plane, nx, ny, res, rb, NULL, NULL, ci, NULL, NULL, NULL, NULL);
        o_inflate(ci, nx, ny, K, O_RMAX, R, cT + k * plane);
        free(ci);
    }
    return R;
}

/* Sec. III-C and Eqs. (7)-(9).  A traversable cell (c^T < c^B) of slice k is
 * unique when it differs from the slice below (higher ground or lower cost)
 * and from the slice above (the slice above has higher ground, or this cell
 * has the lower cost).  Slices with no unique cell are removed.
 * Reading: the text runs the test sequentially - once a slice is removed the
 * next one is compared with the last slice that was kept - while the slice
 * above is always the next raw slice; a missing neighbour (before the first
 * kept slice, after the last slice) counts as different. */
void o_simplify(const float* eG, const double* cT, int N, int nx, int ny, double cB, uint8_t* keep) {
    const int64_t plane = (int64_t)nx * ny;
    int p = -1;
    for (int k = 0; k < N; ++k) {
        int found = 0;
        for (int64_t c = 0; c < plane && !found; ++c) {
            double ck = cT[k * plane + c];
            if (!(ck < cB)) continue;
            double ek = eG[k * plane + c];
            int lower = p < 0 || ek > (double)eG[p * plane + c] || ck < cT[p * plane + c];
            int upper = k == N - 1 || (double)eG[(k + 1) * plane + c] > ek || ck < cT[(k + 1) * plane + c];
            found = lower && upper;
        }
        keep[k] = (uint8_t)found;
        if (found) p = k;
    }
}

/* ------------------------------------------------------------------------ */
/* Envelope for comparing an FP32 evaluation with this FP64 one.
 *
 * Eqs. (1)-(4) switch between branches at thresholds; an FP32 evaluation
 * can take the other branch when an operand lies within rounding distance of
 * its threshold.  A predicate is ambiguous here when its operand is within
 * tau * max(1, |threshold|) of the threshold.  For each cell the initial cost
 * is computed under every combination of outcomes of its ambiguous
 * predicates (the neighbour count of Eq. (4) ranges over the gentle flags of
 * its ambiguous neighbours) and lo/hi are the extremes; inflation is
 * monotone in c^init, so inflating lo and hi brackets every admissible
 * result.  Returns the number of ambiguous cell-slices. */

static int o_near(double v, double th, double tau) {
    return isfinite(v) && fabs(v - th) <= tau * fmax(1.0, fabs(th));
}

static double o_cinit_forced(const o_cell* o, const o_robot* rb, int pI, int pB, int pS, int pP) {
    const double cB = rb->c_barrier;
    double cI = pI ? cB : fmax(0.0, (double)rb->alpha_d * ((double)rb->d_ref - o->dI));
    double cG;
    if (pB) cG = cB;
    else if (pS) { double t = o->mgrad / (double)rb->theta_s; cG = (double)rb->alpha_s * t * t; }
    else if (pP) { double t = o->mxy / (double)rb->theta_b; cG = (double)rb->alpha_b * t * t; }
    else cG = cB;
    return fmin(cB, cI + cG);
}

int64_t o_eval_envelope(const float* eG, const float* eC, int N, int nx, int ny, double res,
                        const o_robot* rb, double tau, double* lo, double* hi) {
    double K[(2 * O_RMAX + 1) * (2 * O_RMAX + 1)];
    int R = o_kernel(res, rb->d_inf, rb->d_sm, O_RMAX, K);
    if (R < 0) return R;
    const int64_t plane = (int64_t)nx * ny;
    const int kp = o_patch_threshold(rb);
    int64_t amb_total = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : amb_total)
    for (int k = 0; k < N; ++k) {
        const float* g = eG + k * plane;
        const float* c = eC + k * plane;
        double* l = (double*)malloc(sizeof(double) * plane);
        double* u = (double*)malloc(sizeof(double) * plane);
        uint8_t* gamb = (uint8_t*)malloc(plane);
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                double gx, gy, mxy, mg;
                o_slope(g, nx, ny, res, x, y, &gx, &gy, &mxy, &mg);
                gamb[(int64_t)y * nx + x] = isfinite(o_g(g, nx, ny, x, y)) && o_near(mg, rb->theta_s, tau);
            }
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int64_t i = (int64_t)y * nx + x;
                o_cell o = o_eval_cell(g, c, nx, ny, res, rb, x, y);
                l[i] = u[i] = o.cinit;
                if (o.branch == 0) continue;
                int aI = o_near(o.dI, rb->d_min, tau);
                int aB = o_near(o.mxy, rb->theta_b, tau);
                int aS = o_near(o.mgrad, rb->theta_s, tau);
                int namb = 0, rp = rb->patch_radius;
                for (int dy = -rp; dy <= rp; ++dy)
                    for (int dx = -rp; dx <= rp; ++dx) {
                        int qx = x + dx, qy = y + dy;
                        if ((dx || dy) && qx >= 0 && qy >= 0 && qx < nx && qy < ny)
                            namb += gamb[(int64_t)qy * nx + qx];
                    }
                /* count of definitely-gentle neighbours and the ambiguous range */
                int cnt_def = o.count;
                for (int dy = -rp; dy <= rp; ++dy)
                    for (int dx = -rp; dx <= rp; ++dx) {
                        int qx = x + dx, qy = y + dy;
                        if ((dx || dy) && qx >= 0 && qy >= 0 && qx < nx && qy < ny &&
                            gamb[(int64_t)qy * nx + qx] && o_is_gentle(g, nx, ny, res, rb, qx, qy))
                            --cnt_def;
                    }
                int aP = cnt_def <= kp && kp < cnt_def + namb;
                if (!(aI || aB || aS || aP)) continue;
                ++amb_total;
                int vI = o.dI < (double)rb->d_min, vB = o.mxy > (double)rb->theta_b;
                int vS = o.mgrad < (double)rb->theta_s, vP = o.count > kp;
                double mn = INFINITY, mx = -INFINITY;
                for (int bI = 0; bI <= aI; ++bI)
                    for (int bB = 0; bB <= aB; ++bB)
                        for (int bS = 0; bS <= aS; ++bS)
                            for (int bP = 0; bP <= aP; ++bP) {
                                double v = o_cinit_forced(&o, rb, aI ? bI : vI, aB ? bB : vB,
                                                          aS ? bS : vS, aP ? bP : vP);
                                mn = fmin(mn, v);
                                mx = fmax(mx, v);
                            }
                l[i] = mn;
                u[i] = mx;
            }
        o_inflate(l, nx, ny, K, O_RMAX, R, lo + k * plane);
        o_inflate(u, nx, ny, K, O_RMAX, R, hi + k * plane);
        free(l);
        free(u);
        free(gamb);
    }
    return amb_total;
}

/* Three-valued check of a keep list produced elsewhere against the
 * simplification rule, with costs known only to within [lo - tol, hi + tol].
 * Walks the given keep list; at each slice the rule is evaluated with Kleene
 * logic (0 false, 1 true, 2 unknown).  Equal definite costs compare as equal.
 * Returns -1 when every decision is admissible, else the first slice whose
 * decision contradicts a definite outcome. */
static int t_and(int a, int b) { return (a == 0 || b == 0) ? 0 : (a == 1 && b == 1) ? 1 : 2; }
static int t_or(int a, int b) { return (a == 1 || b == 1) ? 1 : (a == 0 && b == 0) ? 0 : 2; }

static int o_less3(double lk, double hk, double lp, double hp, double tol) {
    if (hk < lp - 2 * tol) return 1;
    if (lk > hp + 2 * tol) return 0;
    if (lk == hk && lp == hp && lk == lp) return 0;
    return 2;
}

int o_simplify_check(const float* eG, const double* lo, const double* hi, int N, int nx, int ny,
                     double cB, double tol, const uint8_t* keep) {
    const int64_t plane = (int64_t)nx * ny;
    int p = -1;
    for (int k = 0; k < N; ++k) {
        int U = 0;
        for (int64_t c = 0; c < plane && U != 1; ++c) {
            int64_t ik = k * plane + c;
            int trav = hi[ik] < cB - tol ? 1 : (lo[ik] >= cB ? 0 : 2);
            if (trav == 0) continue;
            double ek = eG[ik];
            int lower = 1;
            if (p >= 0) {
                int64_t ip = p * plane + c;
                lower = t_or(ek > (double)eG[ip], o_less3(lo[ik], hi[ik], lo[ip], hi[ip], tol));
            }
            int upper = 1;
            if (k < N - 1) {
                int64_t iu = (k + 1) * plane + c;
                upper = t_or((double)eG[iu] > ek, o_less3(lo[ik], hi[ik], lo[iu], hi[iu], tol));
            }
            U = t_or(U, t_and(trav, t_and(lower, upper)));
        }
        if ((U == 1 && !keep[k]) || (U == 0 && keep[k])) return k;
        if (keep[k]) p = k;
    }
    return -1;
}

/* ------------------------------------------------------------------------ */
/* Trajectory cost sampling (Sec. III-E, Eq. (11)) and adjoints, in FP64.
 *
 * The trajectory optimisation penalises the travel cost C along the
 * trajectory and the deviation of the body height from Z_ref = e^G + d_ref.
 * Reading: a waypoint (x, y, z) on slice k contributes
 *     f = C_k(x, y) + w_z (z - G_k(x, y) - d_ref)^2
 * where C_k and G_k are cell-centred bilinear interpolations of c^T_k and
 * e^G_k (clamped to the grid edge, with zero slope across the clamp).  The
 * height term is dropped when any of the four ground corners is missing.  A
 * trajectory's cost is the sum over its waypoints.  Waypoints with a
 * non-finite coordinate or a slice outside [0, N) contribute nothing. */

static void o_axis(double q, int n, int* i0, int* i1, double* f, double* dq) {
    if (n == 1) { *i0 = *i1 = 0; *f = 0.0; *dq = 0.0; return; }
    double qc = q;
    int clamped = 0;
    if (q < 0.0) { qc = 0.0; clamped = 1; }
    else if (q > (double)(n - 1)) { qc = (double)(n - 1); clamped = 1; }
    int a = (int)floor(qc);
    if (a > n - 2) a = n - 2;
    *i0 = a;
    *i1 = a + 1;
    *f = qc - a;
    *dq = clamped ? 0.0 : 1.0;
}

typedef struct {
    int ok, hterm;
    int64_t c00, c10, c01, c11;
    double fu, fv, du, dv, C, G, res;
} o_bil;

static o_bil o_bilinear(const double* cT, const float* eG, int N, int nx, int ny, const o_grid* g,
                        const float* wp, int k) {
    o_bil b;
    memset(&b, 0, sizeof b);
    if (k < 0 || k >= N || !isfinite(wp[0]) || !isfinite(wp[1]) || !isfinite(wp[2])) return b;
    b.ok = 1;
    double r = (double)g->res;
    double u = ((double)wp[0] - (double)g->x0) / r - 0.5;
    double v = ((double)wp[1] - (double)g->y0) / r - 0.5;
    int i0, i1, j0, j1;
    o_axis(u, nx, &i0, &i1, &b.fu, &b.du);
    o_axis(v, ny, &j0, &j1, &b.fv, &b.dv);
    b.du /= r;
    b.dv /= r;
    if (nx == 1) i1 = 0;
    if (ny == 1) j1 = 0;
    int64_t base = (int64_t)k * nx * ny;
    b.c00 = base + (int64_t)j0 * nx + i0;
    b.c10 = base + (int64_t)j0 * nx + i1;
    b.c01 = base + (int64_t)j1 * nx + i0;
    b.c11 = base + (int64_t)j1 * nx + i1;
    double w00 = (1 - b.fu) * (1 - b.fv), w10 = b.fu * (1 - b.fv), w01 = (1 - b.fu) * b.fv, w11 = b.fu * b.fv;
    b.C = w00 * cT[b.c00] + w10 * cT[b.c10] + w01 * cT[b.c01] + w11 * cT[b.c11];
    b.hterm = isfinite(eG[b.c00]) && isfinite(eG[b.c10]) && isfinite(eG[b.c01]) && isfinite(eG[b.c11]);
    if (b.hterm)
        b.G = w00 * eG[b.c00] + w10 * eG[b.c10] + w01 * eG[b.c01] + w11 * eG[b.c11];
    return b;
}

void o_sample_fwd(const double* cT, const float* eG, int N, int nx, int ny, const o_grid* g, double w_z,
                  double d_ref, const float* wp, const int32_t* slice, int T, int W, double* f) {
    for (int t = 0; t < T; ++t) {
        double acc = 0.0;
        for (int w = 0; w < W; ++w) {
            const float* p = wp + 3 * ((int64_t)t * W + w);
            o_bil b = o_bilinear(cT, eG, N, nx, ny, g, p, slice[(int64_t)t * W + w]);
            if (!b.ok) continue;
            acc += b.C;
            if (b.hterm) {
                double e = (double)p[2] - b.G - d_ref;
                acc += w_z * e * e;
            }
        }
        f[t] = acc;
    }
}

/* Adjoint of o_sample_fwd: gwp [T][W][3] (overwritten), gcT and gG
 * [N][ny][nx] (accumulated). */
void o_sample_bwd(const double* cT, const float* eG, int N, int nx, int ny, const o_grid* g, double w_z,
                  double d_ref, const float* wp, const int32_t* slice, int T, int W, const double* gf,
                  double* gwp, double* gcT, double* gG) {
    for (int t = 0; t < T; ++t)
        for (int w = 0; w < W; ++w) {
            int64_t i = (int64_t)t * W + w;
            const float* p = wp + 3 * i;
            double* gp = gwp + 3 * i;
            gp[0] = gp[1] = gp[2] = 0.0;
            o_bil b = o_bilinear(cT, eG, N, nx, ny, g, p, slice[i]);
            if (!b.ok) continue;
            double s = gf[t];
            double w00 = (1 - b.fu) * (1 - b.fv), w10 = b.fu * (1 - b.fv), w01 = (1 - b.fu) * b.fv, w11 = b.fu * b.fv;
            /* travel cost term */
            double dCdu = (1 - b.fv) * (cT[b.c10] - cT[b.c00]) + b.fv * (cT[b.c11] - cT[b.c01]);
            double dCdv = (1 - b.fu) * (cT[b.c01] - cT[b.c00]) + b.fu * (cT[b.c11] - cT[b.c10]);
            gp[0] += s * dCdu * b.du;
            gp[1] += s * dCdv * b.dv;
            gcT[b.c00] += s * w00;
            gcT[b.c10] += s * w10;
            gcT[b.c01] += s * w01;
            gcT[b.c11] += s * w11;
            if (b.hterm) {
                double e = (double)p[2] - b.G - d_ref;
                double de = 2.0 * w_z * e * s;   /* d/d(z - G) */
                double dGdu = (1 - b.fv) * ((double)eG[b.c10] - eG[b.c00]) + b.fv * ((double)eG[b.c11] - eG[b.c01]);
                double dGdv = (1 - b.fu) * ((double)eG[b.c01] - eG[b.c00]) + b.fu * ((double)eG[b.c11] - eG[b.c10]);
                gp[0] -= de * dGdu * b.du;
                gp[1] -= de * dGdv * b.dv;
                gp[2] += de;
                gG[b.c00] -= de * w00;
                gG[b.c10] -= de * w10;
                gG[b.c01] -= de * w01;
                gG[b.c11] -= de * w11;
            }
        }
}

/* Adjoint of the traversability evaluation (Eqs. (1)-(6)): given dL/dc^T,
 * accumulate dL/de^G and dL/de^C.
 *   inflation: c^T(p) = K(t*) c^init(p + t*) for the maximising tap t*
 *     (first maximum in row-major window order, rows outer), so the
 *     gradient goes to c^init(p + t*) times K(t*);
 *   Eq. (5): passes to c^I and c^G where c^I + c^G < c^B, else stops;
 *   Eq. (1): d c^I / d e^G = alpha_d = -d c^I / d e^C where
 *     alpha_d (d_ref - d^I) > 0 and d^I >= d_min; zero otherwise;
 *   Eqs. (3)-(4): gentle cost alpha_s |g|^2 / theta_s^2 and step cost
 *     alpha_b max(g_x^2, g_y^2) / theta_b^2 (the larger axis; x on a tie)
 *     differentiate through the central differences g = (e+ - e-) / 2r;
 *     barrier branches and the neighbour count have no gradient.
 * `uncertain` (nullable, [N][ny][nx]) marks gradient entries that an FP32
 * evaluation may route differently: the cells touched from a window whose
 * maximum is within tau of a different tap's product, or whose c^init has a
 * predicate, the clip, the interval kink or the step axis within tau. */
static int o_cell_uncertain(const o_cell* o, const o_robot* rb, int namb_gentle, int kp, double tau) {
    if (o->branch == 0) return 0;
    if (o_near(o->dI, rb->d_min, tau) || o_near(o->mxy, rb->theta_b, tau) || o_near(o->mgrad, rb->theta_s, tau))
        return 1;
    if (namb_gentle) return 1;
    (void)kp;
    double s = o->cI + o->cG;
    if (o_near(s, rb->c_barrier, tau)) return 1;
    if (!(o->dI < rb->d_min) && o_near((double)rb->d_ref - o->dI, 0.0, tau)) return 1;
    if (o->branch == 3 && o_near(fabs(o->gx), fabs(o->gy), tau)) return 1;
    return 0;
}

int o_eval_bwd(const float* eG, const float* eC, int N, int nx, int ny, double res, const o_robot* rb,
               const double* gcT, double* gG, double* gC, uint8_t* uncertain, double tau) {
    double K[(2 * O_RMAX + 1) * (2 * O_RMAX + 1)];
    int R = o_kernel(res, rb->d_inf, rb->d_sm, O_RMAX, K);
    if (R < 0) return R;
    const int w = 2 * O_RMAX + 1;
    const int64_t plane = (int64_t)nx * ny;
    const int kp = o_patch_threshold(rb);
    const double cB = rb->c_barrier;
    o_cell* cells = (o_cell*)malloc(sizeof(o_cell) * plane);
    uint8_t* unc = (uint8_t*)malloc(plane);
    for (int k = 0; k < N; ++k) {
        const float* g = eG + k * plane;
        const float* c = eC + k * plane;
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) cells[(int64_t)y * nx + x] = o_eval_cell(g, c, nx, ny, res, rb, x, y);
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                /* ambiguous gentle flags among the patch neighbours */
                int namb = 0, rp = rb->patch_radius;
                for (int dy = -rp; dy <= rp; ++dy)
                    for (int dx = -rp; dx <= rp; ++dx) {
                        int qx = x + dx, qy = y + dy;
                        if ((dx || dy) && qx >= 0 && qy >= 0 && qx < nx && qy < ny) {
                            const o_cell* q = &cells[(int64_t)qy * nx + qx];
                            namb += q->branch != 0 && o_near(q->mgrad, rb->theta_s, tau);
                        }
                    }
                const o_cell* o = &cells[(int64_t)y * nx + x];
                int cnt_near = namb && (o->branch == 3 || o->branch == 4);
                unc[(int64_t)y * nx + x] = (uint8_t)o_cell_uncertain(o, rb, cnt_near, kp, tau);
            }
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int64_t ip = k * plane + (int64_t)y * nx + x;
                double gc = gcT[ip];
                if (gc == 0.0) continue;
                /* the maximising tap (first in window order) and the runner-up */
                double best = -INFINITY, second = -INFINITY;
                int bx = 0, by = 0, sx = -1, sy = -1;
                for (int n = -R; n <= R; ++n)
                    for (int m = -R; m <= R; ++m) {
                        double kw = K[(n + O_RMAX) * w + (m + O_RMAX)];
                        int qx = x + m, qy = y + n;
                        if (kw <= 0.0 || qx < 0 || qy < 0 || qx >= nx || qy >= ny) continue;
                        double v = kw * cells[(int64_t)qy * nx + qx].cinit;
                        if (v > best) {
                            second = best; sx = bx; sy = by;
                            best = v; bx = qx; by = qy;
                        } else if (v > second) {
                            second = v; sx = qx; sy = qy;
                        }
                    }
                double kw = K[(by - y + O_RMAX) * w + (bx - x + O_RMAX)];
                int tie = sx >= 0 && best - second <= tau * fmax(1.0, best) &&
                          !(K[(sy - y + O_RMAX) * w + (sx - x + O_RMAX)] == kw &&
                            cells[(int64_t)sy * nx + sx].cinit == cells[(int64_t)by * nx + bx].cinit);
                const o_cell* q = &cells[(int64_t)by * nx + bx];
                int64_t iq = k * plane + (int64_t)by * nx + bx;
                if (uncertain && (tie || unc[(int64_t)by * nx + bx])) {
                    int pts[2][2] = {{bx, by}, {sx, sy}};
                    for (int a = 0; a < (tie ? 2 : 1); ++a)
                        for (int d = 0; d < 5; ++d) {
                            int ux = pts[a][0] + (d == 1) - (d == 2), uy = pts[a][1] + (d == 3) - (d == 4);
                            if (ux >= 0 && uy >= 0 && ux < nx && uy < ny) uncertain[k * plane + (int64_t)uy * nx + ux] = 1;
                        }
                }
                double gq = kw * gc;
                if (q->branch == 0) continue;
                if (!(q->cI + q->cG < cB)) continue;
                if (!(q->dI < (double)rb->d_min) && (double)rb->alpha_d * ((double)rb->d_ref - q->dI) > 0.0) {
                    gG[iq] += (double)rb->alpha_d * gq;
                    gC[iq] -= (double)rb->alpha_d * gq;
                }
                double dgx = 0.0, dgy = 0.0;   /* dL/dg^x, dL/dg^y */
                if (q->branch == 2) {
                    double ts = rb->theta_s;
                    dgx = 2.0 * rb->alpha_s * q->gx / (ts * ts) * gq;
                    dgy = 2.0 * rb->alpha_s * q->gy / (ts * ts) * gq;
                } else if (q->branch == 3) {
                    double tb = rb->theta_b;
                    if (fabs(q->gx) >= fabs(q->gy)) dgx = 2.0 * rb->alpha_b * q->gx / (tb * tb) * gq;
                    else dgy = 2.0 * rb->alpha_b * q->gy / (tb * tb) * gq;
                }
                if (dgx != 0.0) {
                    gG[iq + 1] += dgx / (2.0 * res);
                    gG[iq - 1] -= dgx / (2.0 * res);
                }
                if (dgy != 0.0) {
                    gG[iq + nx] += dgy / (2.0 * res);
                    gG[iq - nx] -= dgy / (2.0 * res);
                }
            }
    }
    free(cells);
    free(unc);
    return R;
}

/* Adjoint of the construction: each stored ground or ceiling value is the
 * height of one point (its recorded id), so its gradient is added to that
 * point's z.  gz [n] is accumulated. */
void o_route(const double* gG, const double* gC, const int32_t* aG, const int32_t* aC, int64_t ncs, int64_t n,
             double* gz) {
    for (int64_t i = 0; i < ncs; ++i) {
        if (aG[i] >= 0 && aG[i] < n) gz[aG[i]] += gG[i];
        if (aC[i] >= 0 && aC[i] < n) gz[aC[i]] += gC[i];
    }
}

/* Discrete decisions of the evaluation per cell-slice, for finite-difference
 * checks (a central difference is exact when no decision changes inside the
 * step): bits 0-2 the Eq. (1)-(4) branch of c^init, bit 3 the Eq. (5) clip,
 * bits 4-5 the regime of c^I (barrier / positive / zero), bit 6 the step
 * axis, bits 8.. the maximising tap of the inflation window. */
int o_eval_signature(const float* eG, const float* eC, int N, int nx, int ny, double res, const o_robot* rb,
                     int32_t* sig) {
    double K[(2 * O_RMAX + 1) * (2 * O_RMAX + 1)];
    int R = o_kernel(res, rb->d_inf, rb->d_sm, O_RMAX, K);
    if (R < 0) return R;
    const int w = 2 * O_RMAX + 1;
    const int64_t plane = (int64_t)nx * ny;
    o_cell* cells = (o_cell*)malloc(sizeof(o_cell) * plane);
    for (int k = 0; k < N; ++k) {
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x)
                cells[(int64_t)y * nx + x] = o_eval_cell(eG + k * plane, eC + k * plane, nx, ny, res, rb, x, y);
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const o_cell* o = &cells[(int64_t)y * nx + x];
                int code = o->branch;
                if (o->branch) {
                    code |= (o->cI + o->cG >= rb->c_barrier) << 3;
                    int reg = o->dI < (double)rb->d_min ? 0 : ((double)rb->d_ref - o->dI > 0.0 ? 1 : 2);
                    code |= reg << 4;
                    code |= (o->branch == 3 && !(fabs(o->gx) >= fabs(o->gy))) << 6;
                }
                double best = -INFINITY;
                int arg = 0, idx = 0;
                for (int n = -R; n <= R; ++n)
                    for (int m = -R; m <= R; ++m, ++idx) {
                        double kw = K[(n + O_RMAX) * w + (m + O_RMAX)];
                        int qx = x + m, qy = y + n;
                        if (kw <= 0.0 || qx < 0 || qy < 0 || qx >= nx || qy >= ny) continue;
                        double v = kw * cells[(int64_t)qy * nx + qx].cinit;
                        if (v > best) { best = v; arg = idx; }
                    }
                sig[k * plane + (int64_t)y * nx + x] = code | (arg << 8);
            }
    }
    free(cells);
    return R;
}

/* ------------------------------------------------------------------------ */
/* Sec. III-D: path search through the tomogram slices.
 *
 * The search runs on L layers (the slices kept by the simplification, in
 * increasing order), given as c^T and e^G arrays [L][ny][nx] in FP32.
 * The graph, as the section describes it:
 *   - a node is a cell (x, y) of a layer l; it links to its eight planar
 *     neighbours on the same layer;
 *   - the layers directly above and below are checked at the same cell: a
 *     layer whose ground elevation is equal is the same point in space, and
 *     the node cost c^N is the least c^T among the node and those layers;
 *   - moving onto a node v costs c^N(v) plus the length of the step; a node
 *     with c^N = c^B cannot be entered;
 *   - if the layer above has the same ground and a strictly lower c^T, the
 *     node is a gateway to it (moving up costs nothing: it is the same point);
 *     the same holds downwards.
 * Readings where the section is silent: the step length is measured in
 * cells (1 straight, sqrt 2 diagonal, the planar Euclidean distance; the
 * diagonal-distance heuristic uses the same unit); diagonal steps need no free
 * orthogonal neighbours; the start node may itself be a barrier.
 * A* with the diagonal-distance heuristic (admissible and consistent here,
 * since every step costs at least its length) finds a least-cost path; its
 * cost is the shortest-path distance, which this function computes for every
 * node by Dijkstra's algorithm.  Distances are FP64 sums, each edge cost
 * (double)c^N + step length, added to the distance of its tail; unreachable
 * nodes get +inf. */

static double o_node_cost(const float* cT, const float* eG, int L, int64_t plane, int l, int64_t c) {
    double cn = cT[l * plane + c];
    if (l + 1 < L && eG[(l + 1) * plane + c] == eG[l * plane + c] && cT[(l + 1) * plane + c] < cn)
        cn = cT[(l + 1) * plane + c];
    if (l > 0 && eG[(l - 1) * plane + c] == eG[l * plane + c] && cT[(l - 1) * plane + c] < cn)
        cn = cT[(l - 1) * plane + c];
    return cn;
}

/* gateway from layer l to layer m = l +- 1 at cell c */
static int o_gateway(const float* cT, const float* eG, int L, int64_t plane, int l, int m, int64_t c) {
    if (m < 0 || m >= L) return 0;
    return eG[m * plane + c] == eG[l * plane + c] && cT[m * plane + c] < cT[l * plane + c];
}

typedef struct {
    double d;
    int64_t v;
} o_hitem;

static void o_heap_push(o_hitem* h, int64_t* n, double d, int64_t v) {
    int64_t i = (*n)++;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (h[p].d <= d) break;
        h[i] = h[p];
        i = p;
    }
    h[i].d = d;
    h[i].v = v;
}

static o_hitem o_heap_pop(o_hitem* h, int64_t* n) {
    o_hitem top = h[0], last = h[--(*n)];
    int64_t i = 0;
    for (;;) {
        int64_t a = 2 * i + 1;
        if (a >= *n) break;
        if (a + 1 < *n && h[a + 1].d < h[a].d) ++a;
        if (h[a].d >= last.d) break;
        h[i] = h[a];
        i = a;
    }
    if (*n > 0) h[i] = last;
    return top;
}

static const int o_dx8[8] = {-1, 0, 1, -1, 1, -1, 0, 1};
static const int o_dy8[8] = {-1, -1, -1, 0, 0, 1, 1, 1};

/* Returns the number of nodes settled, or -1 on a bad start / no memory. */
int64_t o_plan(const float* cT, const float* eG, int L, int nx, int ny, double cB, int sx, int sy, int sl,
               double* dist) {
    const int64_t plane = (int64_t)nx * ny, nn = (int64_t)L * plane;
    if (sx < 0 || sy < 0 || sl < 0 || sx >= nx || sy >= ny || sl >= L) return -1;
    const double diag = sqrt(2.0);
    for (int64_t v = 0; v < nn; ++v) dist[v] = INFINITY;
    /* each node enters the heap at most once per in-edge: 10 per node */
    o_hitem* h = (o_hitem*)malloc(sizeof(o_hitem) * (size_t)(10 * nn + 1));
    uint8_t* done = (uint8_t*)calloc((size_t)nn, 1);
    if (!h || !done) {
        free(h);
        free(done);
        return -1;
    }
    int64_t n = 0, settled = 0;
    const int64_t s = (int64_t)sl * plane + (int64_t)sy * nx + sx;
    dist[s] = 0.0;
    o_heap_push(h, &n, 0.0, s);
    while (n > 0) {
        o_hitem it = o_heap_pop(h, &n);
        const int64_t u = it.v;
        if (done[u]) continue;
        done[u] = 1;
        ++settled;
        const int l = (int)(u / plane);
        const int64_t c = u % plane;
        const int x = (int)(c % nx), y = (int)(c / nx);
        for (int e = 0; e < 8; ++e) {
            const int x2 = x + o_dx8[e], y2 = y + o_dy8[e];
            if (x2 < 0 || y2 < 0 || x2 >= nx || y2 >= ny) continue;
            const int64_t c2 = (int64_t)y2 * nx + x2;
            const double cn = o_node_cost(cT, eG, L, plane, l, c2);
            if (!(cn < cB)) continue;
            const double w = cn + ((o_dx8[e] != 0 && o_dy8[e] != 0) ? diag : 1.0);
            const double nd = dist[u] + w;
            const int64_t v = (int64_t)l * plane + c2;
            if (nd < dist[v]) {
                dist[v] = nd;
                o_heap_push(h, &n, nd, v);
            }
        }
        for (int m = l - 1; m <= l + 1; m += 2) {
            if (!o_gateway(cT, eG, L, plane, l, m, c)) continue;
            const int64_t v = (int64_t)m * plane + c;
            const double nd = dist[u] + 0.0;
            if (nd < dist[v]) {
                dist[v] = nd;
                o_heap_push(h, &n, nd, v);
            }
        }
    }
    free(h);
    free(done);
    return settled;
}

/* A least-cost path from the start to the goal, read back from the
 * distances: from the goal, step to the first predecessor u (in the order:
 * gateway from the layer below, gateway from the layer above, then the eight
 * planar neighbours in row-major order of (dy, dx)) whose distance plus the
 * edge cost equals the node's distance, until the start.  path receives
 * (x, y, layer) triples from start to goal.  Returns the node count, 0 if the
 * goal is unreachable, -1 on a bad argument, -2 if max_len is too small. */
int o_plan_path(const float* cT, const float* eG, int L, int nx, int ny, double cB, const double* dist, int sx,
                int sy, int sl, int gx, int gy, int gl, int32_t* path, int max_len) {
    const int64_t plane = (int64_t)nx * ny;
    if (sx < 0 || sy < 0 || sl < 0 || sx >= nx || sy >= ny || sl >= L) return -1;
    if (gx < 0 || gy < 0 || gl < 0 || gx >= nx || gy >= ny || gl >= L) return -1;
    const double diag = sqrt(2.0);
    int64_t v = (int64_t)gl * plane + (int64_t)gy * nx + gx;
    const int64_t s = (int64_t)sl * plane + (int64_t)sy * nx + sx;
    if (!(dist[v] < INFINITY)) return 0;
    int len = 0;
    for (;;) {
        if (len >= max_len) return -2;
        const int l = (int)(v / plane);
        const int64_t c = v % plane;
        const int x = (int)(c % nx), y = (int)(c / nx);
        path[3 * len] = x;
        path[3 * len + 1] = y;
        path[3 * len + 2] = l;
        ++len;
        if (v == s) break;
        int64_t u = -1;
        for (int m = l - 1; m <= l + 1 && u < 0; m += 2) {
            if (m < 0 || m >= L) continue;
            if (o_gateway(cT, eG, L, plane, m, l, c) && dist[(int64_t)m * plane + c] + 0.0 == dist[v])
                u = (int64_t)m * plane + c;
        }
        const double cn = o_node_cost(cT, eG, L, plane, l, c);
        for (int e = 0; e < 8 && u < 0 && cn < cB; ++e) {
            const int x2 = x + o_dx8[e], y2 = y + o_dy8[e];
            if (x2 < 0 || y2 < 0 || x2 >= nx || y2 >= ny) continue;
            const int64_t u2 = (int64_t)l * plane + (int64_t)y2 * nx + x2;
            const double w = cn + ((o_dx8[e] != 0 && o_dy8[e] != 0) ? diag : 1.0);
            if (dist[u2] + w == dist[v]) u = u2;
        }
        if (u < 0) return -1; /* not a distance field of this graph */
        v = u;
    }
    for (int a = 0, b = len - 1; a < b; ++a, --b)
        for (int t = 0; t < 3; ++t) {
            int32_t tmp = path[3 * a + t];
            path[3 * a + t] = path[3 * b + t];
            path[3 * b + t] = tmp;
        }
    return len;
}

/* ------------------------------------------------------------------------ */
/* Sec. III-C, closing remark: the simplified tomogram stored sparsely, as
 * the unique cells of the kept slices only.  For kept slice k, with p the
 * last kept slice below it (none for the first), cell c is unique when
 * (Eqs. (8)-(9)) c^T_k < c^B, and (p is none, or e_k > e_p, or
 * c_k < c_p), and (k is the last slice, or e_{k+1} > e_k, or c_k < c_{k+1}).
 * Slices are taken in increasing order and cells in raster order; each
 * unique cell is stored as its cell index and its e^G, e^C, c^T.  Here c^T
 * is FP32 (the comparisons are exact either way).  slice_off [N+1] receives
 * the start of each slice's run (removed slices have empty runs).  Returns
 * the number of unique cells; arrays are written only up to capacity. */
int64_t o_unique_cells(const float* eG, const float* eC, const float* cT, int N, int nx, int ny, double cB,
                       const uint8_t* keep, int64_t capacity, int32_t* cell, float* g_out, float* c_out,
                       float* t_out, int64_t* slice_off) {
    const int64_t plane = (int64_t)nx * ny;
    int64_t m = 0;
    int p = -1;
    for (int k = 0; k < N; ++k) {
        slice_off[k] = m;
        if (!keep[k]) continue;
        for (int64_t c = 0; c < plane; ++c) {
            const double ck = cT[k * plane + c];
            if (!(ck < cB)) continue;
            const double ek = eG[k * plane + c];
            int lower = p < 0 || ek > (double)eG[p * plane + c] || ck < (double)cT[p * plane + c];
            int upper = k == N - 1 || (double)eG[(k + 1) * plane + c] > ek || ck < (double)cT[(k + 1) * plane + c];
            if (!(lower && upper)) continue;
            if (m < capacity) {
                cell[m] = (int32_t)c;
                g_out[m] = eG[k * plane + c];
                c_out[m] = eC[k * plane + c];
                t_out[m] = cT[k * plane + c];
            }
            ++m;
        }
        p = k;
    }
    slice_off[N] = m;
    return m;
}
