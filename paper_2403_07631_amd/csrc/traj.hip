// Trajectory optimisation through the tomogram (Sec. III-E, Eq. (10)), FP64.
//
// A trajectory is M quintic pieces per axis between fixed start and goal
// states (position, velocity, acceleration).  The variables are the interior
// waypoints and the log-durations tau_i (T_i = exp(tau_i)).  For given
// variables the pieces are the minimum-jerk spline through the waypoints.
// Written with each knot's position, velocity and acceleration (quintic
// Hermite pieces, continuous in derivatives 0..2 by construction), the jerk
// effort is a quadratic form in the interior knots' velocities and
// accelerations; its minimum solves a symmetric block-tridiagonal system
// with 2 x 2 blocks, one block row per interior knot.  That minimum is the
// spline continuous in derivatives 0..4 (so 0..3, as Eq. (10) asks).
//
// Eq. (10)'s constraints enter as penalties sampled at K + 1 evenly spaced
// times per piece, with trapezoid weights T_i / K halved at the ends: the
// height reference Z_ref = e^G + d_ref (squared), and cubic penalties on the
// travel cost above C_safe, on speed and acceleration above their limits,
// on a body below e^G + d_min and above the ceiling e^C.  Maps are the
// piece's slice, interpolated bilinearly at cell centres and clamped to the
// grid edge (zero slope across the clamp); terms that use e^G are dropped
// where a ground corner is missing, the ceiling term where a ceiling corner
// is open, all map terms where the slice lies outside [0, N).
//
// The gradient with respect to the waypoints and durations: the partial
// derivatives at fixed knot states, plus one adjoint solve with the same
// factors (the matrix is symmetric) for the dependence of the solved knot
// states on the variables.  The optimiser is gradient descent with Armijo
// backtracking (sufficient decrease 1e-4, up to 30 halvings, the step
// doubled after each accepted iteration); a failed search ends the run, and
// a trial point with a non-finite duration or sample is rejected.
//
// One wavefront per trajectory, its state in LDS.  Lanes work on the pieces,
// several lanes per piece when M is small (they split the samples and their
// sums are combined by butterfly shuffles); the two block-tridiagonal solves
// run on three lanes, one per axis.
#include "traj_internal.h"

namespace pct {

namespace {

// On the unit interval, the quintic with end data x = (p0, v0, a0, p1, v1,
// a1) has the monomial coefficients c0 = p0, c1 = v0, c2 = a0 / 2 and the
// rows below for c3, c4, c5 (the inverse of the 6 x 6 end-condition
// system).  Its jerk effort is x^T Qhat x, Qhat = B^T W B with W the Gram
// matrix of the monomials' third derivatives on [0, 1].  A piece of duration
// T is the unit piece in scaled time: with e = (0, 1, 2, 0, 1, 2), entry a of
// x is scaled by T^e_a, coefficient j is divided by T^j, and the effort is
// divided by T^5, so Q(T)_ab = Qhat_ab T^(e_a + e_b - 5).
__constant__ double kB[3][6] = {
    {-10.0, -6.0, -1.5, 10.0, -4.0, 0.5},
    {15.0, 8.0, 1.5, -15.0, 7.0, -1.0},
    {-6.0, -3.0, -0.5, 6.0, -3.0, 0.5},
};
__constant__ double kQ[6][6] = {
    {720.0, 360.0, 60.0, -720.0, 360.0, -60.0},
    {360.0, 192.0, 36.0, -360.0, 168.0, -24.0},
    {60.0, 36.0, 9.0, -60.0, 24.0, -3.0},
    {-720.0, -360.0, -60.0, 720.0, -360.0, 60.0},
    {360.0, 168.0, 24.0, -360.0, 192.0, -36.0},
    {-60.0, -24.0, -3.0, 60.0, -36.0, 9.0},
};

__device__ __forceinline__ int hexp(int a) { return a % 3; }

// pw[k + 6] = T^k for k = -6 .. 2
struct Pow {
    double v[9];
    __device__ __forceinline__ double operator()(int k) const { return v[k + 6]; }
};

__device__ __forceinline__ Pow powers(double T) {
    Pow p;
    const double ti = 1.0 / T;
    p.v[6] = 1.0;
    p.v[7] = T;
    p.v[8] = T * T;
    p.v[5] = ti;
    #pragma unroll
    for (int k = 4; k >= 0; --k) p.v[k] = p.v[k + 1] * ti;
    return p;
}

__device__ __forceinline__ double qel(const Pow& p, int a, int b) { return kQ[a][b] * p(hexp(a) + hexp(b) - 5); }

// The wavefront's state in LDS, laid out for its M pieces (M + 1 knots).
struct Smem {
    double *T, *tau;
    double (*P)[3], (*V)[3], (*A)[3];
    double (*Dinv)[4], (*Fm)[4], (*Um)[4];  // block factors per interior knot
    double (*rp)[2][3];                     // forward-eliminated right-hand sides
    double (*lam)[2][3];                    // adjoint per interior knot
    double (*gx)[6][3];                     // d(effort + penalties) / d(piece end data)
    double *gT;                             // ... / d T_i at fixed end data
    double *val;
    double (*xk)[3], *xt;  // accepted variables
    double (*gk)[3], *gt;  // gradient there
};

__host__ __device__ constexpr int smem_doubles(int M) {
    return 2 * M + 3 * 3 * (M + 1) + 3 * 4 * M + 6 * M + 6 * (M + 1) + 18 * M + 2 * M + 4 * M + 4 * M;
}

__device__ __forceinline__ Smem smem_view(double* base, int M) {
    Smem s;
    double* p = base;
    auto take = [&](int n) {
        double* q = p;
        p += n;
        return q;
    };
    s.T = take(M);
    s.tau = take(M);
    s.P = (double(*)[3])take(3 * (M + 1));
    s.V = (double(*)[3])take(3 * (M + 1));
    s.A = (double(*)[3])take(3 * (M + 1));
    s.Dinv = (double(*)[4])take(4 * M);
    s.Fm = (double(*)[4])take(4 * M);
    s.Um = (double(*)[4])take(4 * M);
    s.rp = (double(*)[2][3])take(6 * M);
    s.lam = (double(*)[2][3])take(6 * (M + 1));
    s.gx = (double(*)[6][3])take(18 * M);
    s.gT = take(M);
    s.val = take(M);
    s.xk = (double(*)[3])take(3 * M);
    s.xt = take(M);
    s.gk = (double(*)[3])take(3 * M);
    s.gt = take(M);
    return s;
}

__device__ __forceinline__ void inv2(const double m[4], double o[4]) {
    const double det = m[0] * m[3] - m[1] * m[2];
    const double id = 1.0 / det;
    o[0] = m[3] * id;
    o[1] = -m[1] * id;
    o[2] = -m[2] * id;
    o[3] = m[0] * id;
}

__device__ __forceinline__ void mul2(const double a[4], const double b[4], double o[4]) {
    o[0] = a[0] * b[0] + a[1] * b[2];
    o[1] = a[0] * b[1] + a[1] * b[3];
    o[2] = a[2] * b[0] + a[3] * b[2];
    o[3] = a[2] * b[1] + a[3] * b[3];
}

// Interior knot states of the minimum-jerk spline: lanes 0..2 (one axis
// each) eliminate forward; lane 0 keeps the factors for the back pass and
// the adjoint.
__device__ __forceinline__ void solve_knots(const Smem& s, int M) {
    const int ax = threadIdx.x;
    if (ax < 3) {
        double Dp[4] = {0, 0, 0, 0}, Up[4] = {0, 0, 0, 0}, rprev[2] = {0, 0};
        for (int m = 1; m < M; ++m) {
            const Pow pl = powers(s.T[m - 1]), pr = powers(s.T[m]);
            double D[4], L[4], U[4], r[2];
            #pragma unroll
            for (int i = 0; i < 2; ++i) {
                #pragma unroll
                for (int j = 0; j < 2; ++j) {
                    D[2 * i + j] = qel(pl, 4 + i, 4 + j) + qel(pr, 1 + i, 1 + j);
                    L[2 * i + j] = qel(pl, 4 + i, 1 + j);
                    U[2 * i + j] = qel(pr, 1 + i, 4 + j);
                }
                double b = qel(pl, 4 + i, 0) * s.P[m - 1][ax] + qel(pl, 4 + i, 3) * s.P[m][ax] +
                           qel(pr, 1 + i, 0) * s.P[m][ax] + qel(pr, 1 + i, 3) * s.P[m + 1][ax];
                if (m == 1) b += qel(pl, 4 + i, 1) * s.V[0][ax] + qel(pl, 4 + i, 2) * s.A[0][ax];
                if (m == M - 1) b += qel(pr, 1 + i, 4) * s.V[M][ax] + qel(pr, 1 + i, 5) * s.A[M][ax];
                r[i] = -b;
            }
            double F[4] = {0, 0, 0, 0};
            if (m >= 2) {
                mul2(L, Dp, F);
                double FU[4];
                mul2(F, Up, FU);
                #pragma unroll
                for (int q = 0; q < 4; ++q) D[q] -= FU[q];
                r[0] -= F[0] * rprev[0] + F[1] * rprev[1];
                r[1] -= F[2] * rprev[0] + F[3] * rprev[1];
            }
            double Di[4];
            inv2(D, Di);
            if (ax == 0) {
                #pragma unroll
                for (int q = 0; q < 4; ++q) {
                    s.Dinv[m][q] = Di[q];
                    s.Fm[m][q] = F[q];
                    s.Um[m][q] = U[q];
                }
            }
            s.rp[m][0][ax] = r[0];
            s.rp[m][1][ax] = r[1];
            #pragma unroll
            for (int q = 0; q < 4; ++q) {
                Dp[q] = Di[q];
                Up[q] = U[q];
            }
            rprev[0] = r[0];
            rprev[1] = r[1];
        }
    }
    __syncthreads();
    if (ax < 3) {
        double z[2] = {0, 0};
        for (int m = M - 1; m >= 1; --m) {
            double r0 = s.rp[m][0][ax], r1 = s.rp[m][1][ax];
            if (m < M - 1) {
                r0 -= s.Um[m][0] * z[0] + s.Um[m][1] * z[1];
                r1 -= s.Um[m][2] * z[0] + s.Um[m][3] * z[1];
            }
            z[0] = s.Dinv[m][0] * r0 + s.Dinv[m][1] * r1;
            z[1] = s.Dinv[m][2] * r0 + s.Dinv[m][3] * r1;
            s.V[m][ax] = z[0];
            s.A[m][ax] = z[1];
        }
    }
    __syncthreads();
}

// The adjoint: H lambda = d(effort + penalties) / d(interior knot
// velocities and accelerations), with the factors of solve_knots.
__device__ __forceinline__ void solve_adjoint(const Smem& s, int M) {
    const int ax = threadIdx.x;
    if (ax < 3) {
        double prev[2] = {0, 0};
        for (int m = 1; m < M; ++m) {
            double r0 = s.gx[m - 1][4][ax] + s.gx[m][1][ax];
            double r1 = s.gx[m - 1][5][ax] + s.gx[m][2][ax];
            if (m >= 2) {
                r0 -= s.Fm[m][0] * prev[0] + s.Fm[m][1] * prev[1];
                r1 -= s.Fm[m][2] * prev[0] + s.Fm[m][3] * prev[1];
            }
            s.rp[m][0][ax] = r0;
            s.rp[m][1][ax] = r1;
            prev[0] = r0;
            prev[1] = r1;
        }
        double z[2] = {0, 0};
        for (int m = M - 1; m >= 1; --m) {
            double r0 = s.rp[m][0][ax], r1 = s.rp[m][1][ax];
            if (m < M - 1) {
                r0 -= s.Um[m][0] * z[0] + s.Um[m][1] * z[1];
                r1 -= s.Um[m][2] * z[0] + s.Um[m][3] * z[1];
            }
            z[0] = s.Dinv[m][0] * r0 + s.Dinv[m][1] * r1;
            z[1] = s.Dinv[m][2] * r0 + s.Dinv[m][3] * r1;
            s.lam[m][0][ax] = z[0];
            s.lam[m][1][ax] = z[1];
        }
    }
    __syncthreads();
}

// Clamped cell-centred coordinate along one axis.
__device__ __forceinline__ void axis_of(double q, int n, double rinv, int& i0, int& i1, double& f, double& d) {
    if (n == 1) {
        i0 = i1 = 0;
        f = 0.0;
        d = 0.0;
        return;
    }
    double qc = q;
    d = rinv;
    if (q < 0.0) {
        qc = 0.0;
        d = 0.0;
    } else if (q > (double)(n - 1)) {
        qc = (double)(n - 1);
        d = 0.0;
    }
    int a = (int)floor(qc);
    if (a > n - 2) a = n - 2;
    i0 = a;
    i1 = a + 1;
    f = qc - a;
}

struct Bil {
    double v, dx, dy;
    bool ok;
};

__device__ __forceinline__ Bil bilinear(const float* __restrict__ g, long long o00, long long o10, long long o01,
                                        long long o11, double fu, double fv, double du, double dv) {
    Bil b;
    const double g00 = g[o00], g10 = g[o10], g01 = g[o01], g11 = g[o11];
    b.ok = isfinite(g00) && isfinite(g10) && isfinite(g01) && isfinite(g11);
    b.v = b.dx = b.dy = 0.0;
    if (b.ok) {
        b.v = (1 - fu) * (1 - fv) * g00 + fu * (1 - fv) * g10 + (1 - fu) * fv * g01 + fu * fv * g11;
        b.dx = ((1 - fv) * (g10 - g00) + fv * (g11 - g01)) * du;
        b.dy = ((1 - fu) * (g01 - g00) + fu * (g11 - g10)) * dv;
    }
    return b;
}

__device__ __forceinline__ double pos3(double x) { return x > 0.0 ? x : 0.0; }

// Objective (and with GRAD its gradient) at the variables held in s.P[1..M-1]
// and s.tau.  Returns +inf (uniform over the wavefront) at a point with a
// non-finite duration or sample.
template <bool GRAD>
__device__ __forceinline__ double evaluate(const Smem& s, const TrajArgs& a, int lpp, const int* __restrict__ slice, double* coef_out) {
    const int lane = threadIdx.x;
    const int M = a.M;
    bool bad = false;
    if (lane < M) {
        const double T = exp(s.tau[lane]);
        s.T[lane] = T;
        bad = !(T > 0.0) || !isfinite(T);
    }
    if (__ballot(bad) != 0ull) return INFINITY;
    __syncthreads();
    solve_knots(s, M);

    const int piece = lane / lpp, sub = lane % lpp;
    const bool live = piece < M;
    double F = 0.0, gTp = 0.0;
    double gc[6][3];
    double c[6][3], x[6][3];
    #pragma unroll
    for (int j = 0; j < 6; ++j)
        #pragma unroll
        for (int d = 0; d < 3; ++d) gc[j][d] = 0.0;
    double T = 1.0;
    if (live) {
        T = s.T[piece];
        const Pow pw = powers(T);
        #pragma unroll
        for (int d = 0; d < 3; ++d) {
            x[0][d] = s.P[piece][d];
            x[1][d] = s.V[piece][d];
            x[2][d] = s.A[piece][d];
            x[3][d] = s.P[piece + 1][d];
            x[4][d] = s.V[piece + 1][d];
            x[5][d] = s.A[piece + 1][d];
            c[0][d] = x[0][d];
            c[1][d] = x[1][d];
            c[2][d] = 0.5 * x[2][d];
            #pragma unroll
            for (int j = 3; j < 6; ++j) {
                double acc = 0.0;
                #pragma unroll
                for (int e = 0; e < 6; ++e) acc += kB[j - 3][e] * x[e][d] * pw(hexp(e) - j);
                c[j][d] = acc;
            }
        }
        const int k = slice[piece];
        const bool on_map = k >= 0 && k < a.N;
        const long long base = on_map ? (long long)k * a.nx * a.ny : 0;
        const double rinv = 1.0 / a.res;
        const int K = a.K;
        for (int j = sub; j <= K; j += lpp) {
            const double t = T * j / K;
            const double h = (j == 0 || j == K) ? 0.5 : 1.0;
            const double w = T / K * h;
            double q[3], v[3], ac[3], jk[3];
            bool fin = true;
            #pragma unroll
            for (int d = 0; d < 3; ++d) {
                q[d] = ((((c[5][d] * t + c[4][d]) * t + c[3][d]) * t + c[2][d]) * t + c[1][d]) * t + c[0][d];
                v[d] = (((5.0 * c[5][d] * t + 4.0 * c[4][d]) * t + 3.0 * c[3][d]) * t + 2.0 * c[2][d]) * t + c[1][d];
                ac[d] = ((20.0 * c[5][d] * t + 12.0 * c[4][d]) * t + 6.0 * c[3][d]) * t + 2.0 * c[2][d];
                jk[d] = (60.0 * c[5][d] * t + 24.0 * c[4][d]) * t + 6.0 * c[3][d];
                fin = fin && isfinite(q[d]) && isfinite(v[d]) && isfinite(ac[d]);
            }
            if (!fin) {
                bad = true;
                continue;
            }
            double gq[3] = {0, 0, 0}, gv[3], ga[3];
            const double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
            const double a2 = ac[0] * ac[0] + ac[1] * ac[1] + ac[2] * ac[2];
            const double sv = pos3(v2 - a.v_max2), sa = pos3(a2 - a.a_max2);
            double f = a.w_v * (sv * sv * sv) + a.w_a * (sa * sa * sa);
            #pragma unroll
            for (int d = 0; d < 3; ++d) {
                gv[d] = a.w_v * 3.0 * sv * sv * 2.0 * v[d];
                ga[d] = a.w_a * 3.0 * sa * sa * 2.0 * ac[d];
            }
            if (on_map) {
                int i0, i1, j0, j1;
                double fu, fv, du, dv;
                axis_of((q[0] - a.x0) / a.res - 0.5, a.nx, rinv, i0, i1, fu, du);
                axis_of((q[1] - a.y0) / a.res - 0.5, a.ny, rinv, j0, j1, fv, dv);
                const long long o00 = base + (long long)j0 * a.nx + i0, o10 = base + (long long)j0 * a.nx + i1;
                const long long o01 = base + (long long)j1 * a.nx + i0, o11 = base + (long long)j1 * a.nx + i1;
                const Bil C = bilinear(a.cost, o00, o10, o01, o11, fu, fv, du, dv);
                const double sc = pos3(C.v - a.c_safe);
                f += a.w_c * (sc * sc * sc);
                gq[0] += a.w_c * 3.0 * sc * sc * C.dx;
                gq[1] += a.w_c * 3.0 * sc * sc * C.dy;
                const Bil G = bilinear(a.ground, o00, o10, o01, o11, fu, fv, du, dv);
                if (G.ok) {
                    const double e = q[2] - G.v - a.d_ref;
                    const double sg = pos3(G.v + a.d_min - q[2]);
                    f += a.w_z * (e * e) + a.w_h * (sg * sg * sg);
                    // d/dz and d/dG of both terms
                    const double dz = a.w_z * 2.0 * e - a.w_h * 3.0 * sg * sg;
                    const double dG = -a.w_z * 2.0 * e + a.w_h * 3.0 * sg * sg;
                    gq[2] += dz;
                    gq[0] += dG * G.dx;
                    gq[1] += dG * G.dy;
                }
                const Bil H = bilinear(a.ceil, o00, o10, o01, o11, fu, fv, du, dv);
                if (H.ok) {
                    const double sh = pos3(q[2] - H.v);
                    f += a.w_h * (sh * sh * sh);
                    const double dh = a.w_h * 3.0 * sh * sh;
                    gq[2] += dh;
                    gq[0] -= dh * H.dx;
                    gq[1] -= dh * H.dy;
                }
            }
            F += w * f;
            if (GRAD) {
                double dfdt = 0.0;
                #pragma unroll
                for (int d = 0; d < 3; ++d) dfdt += gq[d] * v[d] + gv[d] * ac[d] + ga[d] * jk[d];
                gTp += f * (h / K) + w * dfdt * ((double)j / K);
                double tp[6];
                tp[0] = 1.0;
                #pragma unroll
                for (int m = 1; m < 6; ++m) tp[m] = tp[m - 1] * t;
                #pragma unroll
                for (int d = 0; d < 3; ++d) {
                    gc[0][d] += w * gq[d];
                    #pragma unroll
                    for (int m = 1; m < 6; ++m) {
                        double g = gq[d] * tp[m] + gv[d] * m * tp[m - 1];
                        if (m >= 2) g += ga[d] * (m * (m - 1)) * tp[m - 2];
                        gc[m][d] += w * g;
                    }
                }
            }
        }
    }
    // combine the lanes of a piece (butterfly over the lane group)
    for (int o = 1; o < lpp; o <<= 1) {
        F += __shfl_xor(F, o, 64);
        if (GRAD) {
            gTp += __shfl_xor(gTp, o, 64);
            #pragma unroll
            for (int j = 0; j < 6; ++j)
                #pragma unroll
                for (int d = 0; d < 3; ++d) gc[j][d] += __shfl_xor(gc[j][d], o, 64);
        }
    }
    if (__ballot(bad) != 0ull) return INFINITY;
    if (live && sub == 0) {
        const Pow pw = powers(T);
        double J = 0.0, dJdT = 0.0, dcdT = 0.0;
        #pragma unroll
        for (int d = 0; d < 3; ++d) {
            #pragma unroll
            for (int e = 0; e < 6; ++e) {
                double qx = 0.0, qtx = 0.0;
                #pragma unroll
                for (int b = 0; b < 6; ++b) {
                    qx += qel(pw, e, b) * x[b][d];
                    qtx += qel(pw, e, b) * (hexp(e) + hexp(b) - 5) * x[b][d];
                }
                J += x[e][d] * qx;
                if (GRAD) {
                    dJdT += x[e][d] * qtx;
                    // d c_j / d x_e at fixed T, then the effort's own gradient
                    double g = 2.0 * qx;
                    if (e == 0) g += gc[0][d];
                    if (e == 1) g += gc[1][d];
                    if (e == 2) g += 0.5 * gc[2][d];
                    #pragma unroll
                    for (int j = 3; j < 6; ++j) g += gc[j][d] * kB[j - 3][e] * pw(hexp(e) - j);
                    s.gx[piece][e][d] = g;
                }
            }
            if (GRAD)
                #pragma unroll
                for (int j = 3; j < 6; ++j) {
                    double dc = 0.0;
                    #pragma unroll
                    for (int e = 0; e < 6; ++e) dc += kB[j - 3][e] * (hexp(e) - j) * pw(hexp(e) - j - 1) * x[e][d];
                    dcdT += gc[j][d] * dc;
                }
        }
        s.val[piece] = J + F + a.w_T * T;
        if (GRAD) s.gT[piece] = gTp + dJdT / T + dcdT;
        if (coef_out)
            #pragma unroll
            for (int j = 0; j < 6; ++j)
                #pragma unroll
                for (int d = 0; d < 3; ++d) coef_out[((long long)piece * 6 + j) * 3 + d] = c[j][d];
    }
    __syncthreads();
    double phi = 0.0;
    for (int i = 0; i < M; ++i) phi += s.val[i];
    if (!GRAD) return phi;

    solve_adjoint(s, M);
    if (lane < M) {
        const int i = lane;
        const double Ti = s.T[i];
        const Pow pw = powers(Ti);
        double corrT = 0.0;
        #pragma unroll
        for (int d = 0; d < 3; ++d) {
            double lam[6] = {0, 0, 0, 0, 0, 0};
            if (i >= 1) {
                lam[1] = s.lam[i][0][d];
                lam[2] = s.lam[i][1][d];
            }
            if (i + 1 <= M - 1) {
                lam[4] = s.lam[i + 1][0][d];
                lam[5] = s.lam[i + 1][1][d];
            }
            const double xe[6] = {s.P[i][d], s.V[i][d], s.A[i][d], s.P[i + 1][d], s.V[i + 1][d], s.A[i + 1][d]};
            double c0 = 0.0, c3 = 0.0;
            #pragma unroll
            for (int e = 1; e < 6; ++e) {
                if (e == 3) continue;
                c0 += lam[e] * qel(pw, e, 0);
                c3 += lam[e] * qel(pw, e, 3);
                double st = 0.0;
                #pragma unroll
                for (int b = 0; b < 6; ++b) st += qel(pw, e, b) * (hexp(e) + hexp(b) - 5) * xe[b];
                corrT += lam[e] * st;
            }
            s.gx[i][0][d] -= c0;
            s.gx[i][3][d] -= c3;
        }
        s.gt[i] = Ti * (s.gT[i] - corrT / Ti + a.w_T);
    }
    __syncthreads();
    if (lane >= 1 && lane < M)
        #pragma unroll
        for (int d = 0; d < 3; ++d) s.gk[lane - 1][d] = s.gx[lane - 1][3][d] + s.gx[lane][0][d];
    __syncthreads();
    return phi;
}

// OPT = false: one evaluation with gradient (and coefficients); OPT = true:
// `iters` optimiser iterations in place.
template <bool OPT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_traj(TrajArgs a, int lpp, const double* __restrict__ bound,
                                             const int* __restrict__ slice_all, double* __restrict__ knots,
                                             double* __restrict__ tau, double* __restrict__ phi_out,
                                             double* __restrict__ gknots, double* __restrict__ gtau,
                                             double* __restrict__ coef, int iters, double step,
                                             int* __restrict__ iters_done) {
    extern __shared__ double s_traj[];
    const Smem s = smem_view(s_traj, a.M);
    const int tr = blockIdx.x;
    const int lane = threadIdx.x;
    const int M = a.M;
    const double* bd = bound + (long long)tr * 18;
    const int* slice = slice_all + (long long)tr * M;
    double* kn = knots + (long long)tr * (M - 1) * 3;
    double* ta = tau + (long long)tr * M;
    if (lane < 3) {
        s.P[0][lane] = bd[lane];
        s.V[0][lane] = bd[3 + lane];
        s.A[0][lane] = bd[6 + lane];
        s.P[M][lane] = bd[9 + lane];
        s.V[M][lane] = bd[12 + lane];
        s.A[M][lane] = bd[15 + lane];
    }
    if (lane >= 1 && lane < M)
        #pragma unroll
        for (int d = 0; d < 3; ++d) s.P[lane][d] = kn[(lane - 1) * 3 + d];
    if (lane < M) s.tau[lane] = ta[lane];
    __syncthreads();

    if (!OPT) {
        double* cf = coef ? coef + (long long)tr * M * 18 : nullptr;
        const double phi = evaluate<true>(s, a, lpp, slice, cf);
        if (lane == 0) phi_out[tr] = phi;
        // no gradient at a point with a non-finite duration or sample
        const bool fin = isfinite(phi);
        if (lane >= 1 && lane < M)
            for (int d = 0; d < 3; ++d)
                gknots[(long long)tr * (M - 1) * 3 + (lane - 1) * 3 + d] = fin ? s.gk[lane - 1][d] : NAN;
        if (lane < M) gtau[(long long)tr * M + lane] = fin ? s.gt[lane] : NAN;
        return;
    }

    double phi = evaluate<true>(s, a, lpp, slice, nullptr);
    double alpha = step;
    int done = 0;
    if (isfinite(phi)) {
        if (lane >= 1 && lane < M)
            #pragma unroll
            for (int d = 0; d < 3; ++d) s.xk[lane - 1][d] = s.P[lane][d];
        if (lane < M) s.xt[lane] = s.tau[lane];
        __syncthreads();
        for (int it = 0; it < iters; ++it) {
            double g2 = 0.0;
            for (int i = 0; i < M - 1; ++i)
                #pragma unroll
                for (int d = 0; d < 3; ++d) g2 += s.gk[i][d] * s.gk[i][d];
            for (int i = 0; i < M; ++i) g2 += s.gt[i] * s.gt[i];
            if (g2 == 0.0) break;
            bool ok = false;
            for (int ls = 0; ls < 30; ++ls) {
                __syncthreads();
                if (lane >= 1 && lane < M)
                    #pragma unroll
                    for (int d = 0; d < 3; ++d) s.P[lane][d] = s.xk[lane - 1][d] - alpha * s.gk[lane - 1][d];
                if (lane < M) s.tau[lane] = s.xt[lane] - alpha * s.gt[lane];
                __syncthreads();
                const double pn = evaluate<false>(s, a, lpp, slice, nullptr);
                if (pn <= phi - 1e-4 * alpha * g2) {
                    ok = true;
                    break;
                }
                alpha *= 0.5;
            }
            if (!ok) break;
            __syncthreads();
            if (lane >= 1 && lane < M)
                #pragma unroll
                for (int d = 0; d < 3; ++d) s.xk[lane - 1][d] = s.P[lane][d];
            if (lane < M) s.xt[lane] = s.tau[lane];
            __syncthreads();
            phi = evaluate<true>(s, a, lpp, slice, nullptr);
            alpha *= 2.0;
            ++done;
        }
    }
    __syncthreads();
    if (done > 0) {
        if (lane >= 1 && lane < M)
            #pragma unroll
            for (int d = 0; d < 3; ++d) kn[(lane - 1) * 3 + d] = s.xk[lane - 1][d];
        if (lane < M) ta[lane] = s.xt[lane];
    }
    if (lane == 0) {
        phi_out[tr] = phi;
        if (iters_done) iters_done[tr] = done;
    }
}

}  // namespace

pct_status launch_traj(const TrajArgs& a, int n_traj, const double* bound, const int* slice, double* knots,
                       double* tau, double* phi, double* gknots, double* gtau, double* coef, int iters, double step,
                       int* iters_done, hipStream_t s) {
    if (n_traj == 0) return PCT_OK;
    int lpp = 1;
    while (lpp * 2 * a.M <= 64) lpp *= 2;
    const size_t lds = sizeof(double) * (size_t)smem_doubles(a.M);
    if (iters < 0)
        hipLaunchKernelGGL(k_traj<false>, dim3((unsigned)n_traj), dim3(64), lds, s, a, lpp, bound, slice, knots, tau, phi,
                           gknots, gtau, coef, iters, step, iters_done);
    else
        hipLaunchKernelGGL(k_traj<true>, dim3((unsigned)n_traj), dim3(64), lds, s, a, lpp, bound, slice, knots, tau, phi,
                           gknots, gtau, coef, iters, step, iters_done);
    PCT_LAUNCH_CHECK();
    return PCT_OK;
}

}  // namespace pct
