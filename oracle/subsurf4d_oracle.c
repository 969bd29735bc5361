/*
 * Plain FP64 CPU oracle for the 4D generalized subjective-surface (SUBSURF)
 * segmentation step.  TEST INFRASTRUCTURE ONLY: it exists so that tests,
 * the smoke check and the CPU-baseline leg of the benchmark can check the GPU
 * path against an obviously correct implementation.  The GPU library never
 * links, loads or calls it, and it shares no source with the GPU library.
 *
 * Everything is double precision, written as straight loops in the order the
 * paper states the method, built with -ffp-contract=off so that no multiply-add
 * is fused behind the reader's back.  Speed is not a goal (except that the
 * red-black sweeps accept OpenMP so the CPU baseline can use every host core;
 * the result does not depend on the thread count).
 *
 * Grid conventions (paper Sec. 3.2.2 notation and the 4D-to-1D map of
 * Sec. 3.7): interior cells are i=1..N1, j=1..N2, k=1..N3, l=1..N4; index 0
 * and N+1 are the ghost (boundary) layer; x (i) is the fastest index.  The
 * voxel coordinate of interior cell (i,j,k,l) is X=(i-1,j-1,k-1) in frame l-1.
 * "Padded" arrays hold (N1+2)(N2+2)(N3+2)(N4+2) values, "interior" arrays
 * N1*N2*N3*N4 values, both x-fastest.
 *
 * Face/direction order used for the 8 coefficients of a cell:
 *   0:-x 1:+x 2:-y 3:+y 4:-z 5:+z 6:-t 7:+t
 *
 * Parity: the functions below with a "pinned by" note are checked in tests
 * against closed forms, invariants, a dense direct solve and the paper's
 * convergence table (Sec. 3.4); see tests/test_oracle_*.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    float x, y, z;   /* voxel coordinates of a seed / centre inside frame */
    int32_t frame;   /* 0-based frame index (l-1) */
} oracle_centre;

/* ------------------------------------------------------------------ indexing */

static size_t pidx(const int *n, long i, long j, long k, long l)
{
    const size_t p1 = (size_t)n[0] + 2, p2 = (size_t)n[1] + 2, p3 = (size_t)n[2] + 2;
    return (((size_t)l * p3 + (size_t)k) * p2 + (size_t)j) * p1 + (size_t)i;
}

static size_t iidx(const int *n, long i, long j, long k, long l)
{
    return ((((size_t)l - 1) * n[2] + ((size_t)k - 1)) * n[1] + ((size_t)j - 1)) * n[0] + ((size_t)i - 1);
}

static size_t padded_count(const int *n)
{
    return ((size_t)n[0] + 2) * ((size_t)n[1] + 2) * ((size_t)n[2] + 2) * ((size_t)n[3] + 2);
}

static long clampl(long v, long lo, long hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* unit offset e_d, d = 0..3 for x,y,z,t */
static void unit(int d, long e[4])
{
    e[0] = e[1] = e[2] = e[3] = 0;
    e[d] = 1;
}

/* ------------------------------------------------------ balls and ownership */

/* Squared distance between the voxel centre X=(i-1,j-1,k-1) and a centre, in
 * voxel units (the balls of the local thresholding in Sec. 3.1 and of the
 * local rescaling remark in Sec. 3.2.2 live in one 3D frame). */
static double dist2(const oracle_centre *c, long i, long j, long k)
{
    const double dx = (double)(i - 1) - (double)c->x;
    const double dy = (double)(j - 1) - (double)c->y;
    const double dz = (double)(k - 1) - (double)c->z;
    return dx * dx + dy * dy + dz * dz;
}

/* Bounding box of the ball in 1-based interior indices (one voxel of slack on
 * each side; membership itself is decided by dist2 <= r*r). */
static void ball_box(const int *n, const oracle_centre *c, double r, long lo[3], long hi[3])
{
    const double cc[3] = {c->x, c->y, c->z};
    for (int a = 0; a < 3; ++a) {
        lo[a] = clampl((long)floor(cc[a] - r) + 1 - 1, 1, n[a]);
        hi[a] = clampl((long)ceil(cc[a] + r) + 1 + 1, 1, n[a]);
    }
}

/*
 * Owner map (interior array of int32): for every interior cell the index of the
 * ball B(c_m^l, r) of its own frame that contains it, choosing the nearest
 * centre when several balls contain it (ties -> lowest index), or -1.
 * The paper defines thresholding and rescaling per ball (Sec. 3.1 and the
 * local rescaling remark); overlapping balls are not discussed there, and the
 * nearest-centre owner is this implementation's reading.
 * Pinned by brute force on small inputs (tests/test_oracle_pins.py: owner map and threshold tests).
 */
void oracle_owner_map(const int *n, const oracle_centre *cs, int nc, double r, int32_t *owner)
{
    const size_t ni = (size_t)n[0] * n[1] * n[2] * n[3];
    double *best = (double *)malloc(ni * sizeof(double));
    for (size_t q = 0; q < ni; ++q) { owner[q] = -1; best[q] = 0.0; }
    for (int m = 0; m < nc; ++m) {
        const oracle_centre *c = &cs[m];
        if (c->frame < 0 || c->frame >= n[3]) continue;
        const long l = c->frame + 1;
        long lo[3], hi[3];
        ball_box(n, c, r, lo, hi);
        for (long k = lo[2]; k <= hi[2]; ++k)
            for (long j = lo[1]; j <= hi[1]; ++j)
                for (long i = lo[0]; i <= hi[0]; ++i) {
                    const double d2 = dist2(c, i, j, k);
                    if (!(d2 <= r * r)) continue;
                    const size_t q = iidx(n, i, j, k, l);
                    /* strict '<' keeps the lowest index on ties (m ascends) */
                    if (owner[q] < 0 || d2 < best[q]) { owner[q] = m; best[q] = d2; }
                }
    }
    free(best);
}

/* min and max of an interior field over every ball (paper Sec. 3.1: alpha, beta;
 * local rescaling remark: mu, xi).  Balls that contain no cell get +inf/-inf. */
static void ball_minmax_interior(const int *n, const oracle_centre *cs, int nc, double r,
                                 const double *f, double *mn, double *mx)
{
    for (int m = 0; m < nc; ++m) {
        double lo_v = INFINITY, hi_v = -INFINITY;
        const oracle_centre *c = &cs[m];
        if (c->frame >= 0 && c->frame < n[3]) {
            const long l = c->frame + 1;
            long lo[3], hi[3];
            ball_box(n, c, r, lo, hi);
            for (long k = lo[2]; k <= hi[2]; ++k)
                for (long j = lo[1]; j <= hi[1]; ++j)
                    for (long i = lo[0]; i <= hi[0]; ++i) {
                        if (!(dist2(c, i, j, k) <= r * r)) continue;
                        const double v = f[iidx(n, i, j, k, l)];
                        if (v < lo_v) lo_v = v;
                        if (v > hi_v) hi_v = v;
                    }
        }
        mn[m] = lo_v;
        mx[m] = hi_v;
    }
}

/*
 * Local thresholding (Sec. 3.1, equation of I^TH): per ball,
 *   alpha = min I0, beta = max I0 over the ball,
 *   TH = lambda*alpha + (1-lambda)*beta,
 *   I^TH = beta where I0 >= TH, else alpha    (cells owned by the ball),
 *   I^TH = I0 for cells in no ball (reading: the paper defines I^TH only in balls;
 *   on binary images the paper notes I^TH and I0 coincide).
 * I0 and ITH are interior arrays.  owner from oracle_owner_map.
 */
void oracle_threshold(const int *n, const double *I0, const oracle_centre *cs, int nc, double r,
                      double lambda, const int32_t *owner, double *ITH)
{
    const size_t ni = (size_t)n[0] * n[1] * n[2] * n[3];
    double *alpha = (double *)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(double));
    double *beta = (double *)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(double));
    ball_minmax_interior(n, cs, nc, r, I0, alpha, beta);
    for (size_t q = 0; q < ni; ++q) {
        const int m = owner[q];
        if (m < 0) { ITH[q] = I0[q]; continue; }
        const double th = lambda * alpha[m] + (1.0 - lambda) * beta[m];
        ITH[q] = (I0[q] >= th) ? beta[m] : alpha[m];
    }
    free(alpha);
    free(beta);
}

static double norm2_interior(const int *n, const double *b)
{
    const size_t per = (size_t)n[0] * n[1] * n[2];
    double tot = 0.0;
    for (long l = 0; l < n[3]; ++l) {
        double acc = 0.0;
        for (size_t q = (size_t)l * per; q < (size_t)(l + 1) * per; ++q) acc += b[q] * b[q];
        tot += acc;
    }
    return sqrt(tot);
}

/* ------------------------------------------------------- linear heat (LHE) */

/*
 * One implicit finite-volume step of the 4D linear heat equation with zero
 * Neumann boundary (presmoothing, Sec. 3.1: Gaussian smoothing realised as a
 * heat-equation solve; boundary faces carry no flux):
 *   (1 + tau_s*n_P/h^2) J_P - tau_s/h^2 * sum_{interior nbrs} J_nbr = J_prev,P
 * n_P = number of interior face neighbours of P.  Solved by red-black SOR from
 * the initial guess J_prev until ||b - A J||_2 <= tol ||b||_2 (checked before the
 * first and after every iteration).  Interior arrays.  Returns iterations used,
 * or -1 if max_iter was reached.
 * Pinned by the Neumann cosine eigenmode, mass conservation and constants
 * (tests/test_oracle_pins.py: LHE eigenmode, mass and DMP tests).
 */
static double lhe_row(const int *n, const double *J, const double *rhs, double a, long i, long j,
                      long k, long l, double *diag)
{
    const long c[4] = {i, j, k, l};
    double s = rhs[iidx(n, i, j, k, l)];
    int cnt = 0;
    for (int d = 0; d < 4; ++d) {
        for (int sg = -1; sg <= 1; sg += 2) {
            long q[4] = {c[0], c[1], c[2], c[3]};
            q[d] += sg;
            if (q[d] < 1 || q[d] > n[d]) continue;
            s += a * J[iidx(n, q[0], q[1], q[2], q[3])];
            ++cnt;
        }
    }
    *diag = 1.0 + a * cnt;
    return s;
}

static double lhe_residual2(const int *n, const double *J, const double *rhs, double a)
{
    double tot = 0.0;
    for (long l = 1; l <= n[3]; ++l) {
        double part = 0.0;
        for (long k = 1; k <= n[2]; ++k)
            for (long j = 1; j <= n[1]; ++j)
                for (long i = 1; i <= n[0]; ++i) {
                    double D;
                    const double s = lhe_row(n, J, rhs, a, i, j, k, l, &D);
                    const double r = s - D * J[iidx(n, i, j, k, l)];
                    part += r * r;
                }
        tot += part;
    }
    return tot;
}

int oracle_lhe_step(const int *n, double h, double tau_s, double omega, double tol, int max_iter,
                    const double *Jprev, double *J)
{
    const size_t ni = (size_t)n[0] * n[1] * n[2] * n[3];
    const double a = tau_s / (h * h);
    const double bn = norm2_interior(n, Jprev);
    memcpy(J, Jprev, ni * sizeof(double));
    double R = sqrt(lhe_residual2(n, J, Jprev, a));
    if (R <= tol * bn) return 0;
    for (int it = 1; it <= max_iter; ++it) {
        for (int colour = 0; colour < 2; ++colour) {
#pragma omp parallel for schedule(static)
            for (long l = 1; l <= n[3]; ++l)
                for (long k = 1; k <= n[2]; ++k)
                    for (long j = 1; j <= n[1]; ++j)
                        for (long i = 1; i <= n[0]; ++i) {
                            if (((i + j + k + l) & 1) != colour) continue;
                            double D;
                            const double s = lhe_row(n, J, Jprev, a, i, j, k, l, &D);
                            const size_t q = iidx(n, i, j, k, l);
                            J[q] = omega * (s / D) + (1.0 - omega) * J[q];
                        }
        }
        R = sqrt(lhe_residual2(n, J, Jprev, a));
        if (R <= tol * bn) return it;
    }
    return -1;
}

/* ---------------------------------------------------- reduced diamond cell */

/*
 * Gradient on the "+e_d" face of cell P (the face shared by P and P+e_d),
 * reduced diamond cell in 4D (Sec. 3.2.2, the corner values u^{pq00},... and
 * the face gradients nabla^{p000} u, ...):
 *   normal component     (v[P+e_d] - v[P]) / h
 *   component e != d     (u^{..,+1,..} - u^{..,-1,..}) / h where each corner value
 *                        is the mean of 4 cell values around the corner point, i.e.
 *                        ((v[P]+v[P+e_d]+v[P+e_e]+v[P+e_d+e_e])
 *                         -(v[P]+v[P+e_d]+v[P-e_e]+v[P+e_d-e_e])) / (4h).
 * The "-e_d" face of P is the "+e_d" face of P-e_d (the paper's formulas with
 * p=-1 give the same vector up to the sign of the normal component, so the
 * same norm).  `get` reads v at a (possibly clamped) index.
 * Pinned: exact for every quadratic polynomial (tests/test_oracle_pins.py: face-gradient quadratic test).
 */
typedef double (*getter)(const void *ctx, long i, long j, long k, long l);

static void face_gradient(getter get, const void *ctx, double h, int d, const long P[4], double g[4])
{
    long e[4];
    unit(d, e);
    const long Q[4] = {P[0] + e[0], P[1] + e[1], P[2] + e[2], P[3] + e[3]};
    const double vP = get(ctx, P[0], P[1], P[2], P[3]);
    const double vQ = get(ctx, Q[0], Q[1], Q[2], Q[3]);
    for (int t = 0; t < 4; ++t) {
        if (t == d) { g[t] = (vQ - vP) / h; continue; }
        long f[4];
        unit(t, f);
        const double up = (vP + vQ + get(ctx, P[0] + f[0], P[1] + f[1], P[2] + f[2], P[3] + f[3]) +
                           get(ctx, Q[0] + f[0], Q[1] + f[1], Q[2] + f[2], Q[3] + f[3])) / 4.0;
        const double dn = (vP + vQ + get(ctx, P[0] - f[0], P[1] - f[1], P[2] - f[2], P[3] - f[3]) +
                           get(ctx, Q[0] - f[0], Q[1] - f[1], Q[2] - f[2], Q[3] - f[3])) / 4.0;
        g[t] = (up - dn) / h;
    }
}

typedef struct { const int *n; const double *v; } padded_ctx;
typedef struct { const int *n; const double *v; } clamped_ctx;

static double get_padded(const void *ctx, long i, long j, long k, long l)
{
    const padded_ctx *c = (const padded_ctx *)ctx;
    return c->v[pidx(c->n, i, j, k, l)];
}

/* interior array read with every index clamped to the interior: the ghost of
 * an image is a copy of the nearest interior value (zero-Neumann image). */
static double get_clamped(const void *ctx, long i, long j, long k, long l)
{
    const clamped_ctx *c = (const clamped_ctx *)ctx;
    const int *n = c->n;
    return c->v[iidx(n, clampl(i, 1, n[0]), clampl(j, 1, n[1]), clampl(k, 1, n[2]), clampl(l, 1, n[3]))];
}

/* Face gradients of a padded field on the "+e_d" face of every cell P with
 * 0 <= P_d <= N_d and 1 <= P_t <= N_t for t != d (every face that touches an
 * interior cell); other entries are 0.  out: padded x 4 components. */
void oracle_face_gradient(const int *n, double h, const double *v, int d, double *out)
{
    const size_t np = padded_count(n);
    memset(out, 0, np * 4 * sizeof(double));
    padded_ctx ctx = {n, v};
    for (long l = 0; l <= n[3] + 1; ++l)
        for (long k = 0; k <= n[2] + 1; ++k)
            for (long j = 0; j <= n[1] + 1; ++j)
                for (long i = 0; i <= n[0] + 1; ++i) {
                    const long P[4] = {i, j, k, l};
                    int ok = 1;
                    for (int t = 0; t < 4; ++t) {
                        const long lo = (t == d) ? 0 : 1;
                        if (P[t] < lo || P[t] > n[t]) ok = 0;
                    }
                    if (!ok) continue;
                    double g[4];
                    face_gradient(get_padded, &ctx, h, d, P, g);
                    for (int t = 0; t < 4; ++t) out[pidx(n, i, j, k, l) * 4 + t] = g[t];
                }
}

/*
 * Edge detector on faces (Sec. 3.2.2, the G^{pqrs} equation; g of the
 * Perona-Malik form 1/(1+K s^2), Sec. 2):
 *   G_d(P) = 1 / (1 + K * (delta*|F_d(Is0,P)| + vartheta*|F_d(IsTH,P)|)^2)
 * on the "+e_d" face of every padded cell P (index clamping supplies the image
 * outside the interior).  Is0, IsTH: interior arrays; G: 4 x padded, G[d*np + p].
 * Pinned: constant image -> 1, K=0 -> 1, linear ramp closed form.
 */
void oracle_face_g(const int *n, double h, double K, double delta, double vartheta,
                   const double *Is0, const double *IsTH, double *G)
{
    const size_t np = padded_count(n);
    clamped_ctx c0 = {n, Is0}, c1 = {n, IsTH};
    for (int d = 0; d < 4; ++d)
        for (long l = 0; l <= n[3] + 1; ++l)
            for (long k = 0; k <= n[2] + 1; ++k)
                for (long j = 0; j <= n[1] + 1; ++j)
                    for (long i = 0; i <= n[0] + 1; ++i) {
                        const long P[4] = {i, j, k, l};
                        double g0[4], g1[4];
                        face_gradient(get_clamped, &c0, h, d, P, g0);
                        face_gradient(get_clamped, &c1, h, d, P, g1);
                        const double n0 = sqrt(g0[0] * g0[0] + g0[1] * g0[1] + g0[2] * g0[2] + g0[3] * g0[3]);
                        const double n1 = sqrt(g1[0] * g1[0] + g1[1] * g1[1] + g1[2] * g1[2] + g1[3] * g1[3]);
                        const double s = delta * n0 + vartheta * n1;
                        G[(size_t)d * np + pidx(n, i, j, k, l)] = 1.0 / (1.0 + K * s * s);
                    }
}

/* ------------------------------------------------------ initial condition */

/*
 * Initial segmentation function (Sec. 2, peak profile 1/(|s-x|+v), used per
 * frame in 4D as stated in Sec. 3.1):
 *   R <= 0:  u0 = max over the frame's seeds of 1/(|X-c|+v)
 *   R  > 0:  u0 = max over the frame's seeds of max(0, 1/(|X-c|+v) - 1/(R+v))
 *            (profile cut at radius R and shifted to 0 for zero Dirichlet data)
 * Ghost cells are 0.  u: padded.  Frames without a seed are 0.
 */
void oracle_init_u(const int *n, const oracle_centre *cs, int nc, double v, double R, double *u)
{
    memset(u, 0, padded_count(n) * sizeof(double));
    if (R > 0.0) {
        /* with the cut-off every profile is 0 beyond distance R of its seed, and
         * all values are >= 0: the maximum over the seeds is the maximum over
         * the seeds whose R-ball holds the cell, taken seed by seed over a box
         * around each ball (cells in no ball keep 0) */
        for (int m = 0; m < nc; ++m) {
            const oracle_centre *c = &cs[m];
            if (c->frame < 0 || c->frame >= n[3]) continue;
            const long l = c->frame + 1;
            long lo[3], hi[3];
            ball_box(n, c, R, lo, hi);
            for (long k = lo[2]; k <= hi[2]; ++k)
                for (long j = lo[1]; j <= hi[1]; ++j)
                    for (long i = lo[0]; i <= hi[0]; ++i) {
                        const double dd = sqrt(dist2(c, i, j, k));
                        double val = 1.0 / (dd + v) - 1.0 / (R + v);
                        if (val < 0.0) val = 0.0;
                        double *p = &u[pidx(n, i, j, k, l)];
                        if (val > *p) *p = val;
                    }
        }
        return;
    }
    for (long l = 1; l <= n[3]; ++l)
        for (long k = 1; k <= n[2]; ++k)
            for (long j = 1; j <= n[1]; ++j)
                for (long i = 1; i <= n[0]; ++i) {
                    double best = 0.0;
                    int any = 0;
                    for (int m = 0; m < nc; ++m) {
                        if (cs[m].frame != l - 1) continue;
                        const double dd = sqrt(dist2(&cs[m], i, j, k));
                        const double val = 1.0 / (dd + v);
                        if (!any || val > best) best = val;
                        any = 1;
                    }
                    u[pidx(n, i, j, k, l)] = any ? best : 0.0;
                }
}

/* ------------------------------------------------------------- assembly */

/*
 * Coefficients of the semi-implicit finite-volume system of one time step
 * (Sec. 3.2.2: the system for uniform h, with A_eps and A_eps-bar as printed):
 *   q_f = |grad on face f of w|^2 (reduced diamond cell), f over the 8 faces
 *   A_f = sqrt(eps^2 + q_f)
 *   Abar = sqrt(eps^2 + (1/8) sum_f q_f)
 *   c_f = tau/h^2 * Abar * G_f / A_f
 *   diag = 1 + sum_f c_f
 *   b = w_P + sum over ghost neighbours of c_f * ub_nbr    (Dirichlet data)
 * w: padded u^{resc;n-1} (its ghosts enter the boundary-face gradients);
 * ub: padded array whose ghost values are the Dirichlet data of the new level
 * (ub may equal w); G: 4 x padded face field; coef: interior x 8 (face order
 * -x,+x,-y,+y,-z,+z,-t,+t); b: interior.
 * Pinned: constant preservation, symmetry of c/Abar across each face, the
 * M-matrix properties, the Sec. 3.4 convergence table.
 */
void oracle_assemble(const int *n, double h, double eps, double tau, const double *G,
                     const double *w, const double *ub, double *coef, double *b)
{
    const size_t np = padded_count(n);
    padded_ctx ctx = {n, w};
    const double th2 = tau / (h * h);
#pragma omp parallel for schedule(static)
    for (long l = 1; l <= n[3]; ++l)
        for (long k = 1; k <= n[2]; ++k)
            for (long j = 1; j <= n[1]; ++j)
                for (long i = 1; i <= n[0]; ++i) {
                    const long P[4] = {i, j, k, l};
                    double q[8], Gf[8];
                    long nb[8][4];
                    for (int d = 0; d < 4; ++d) {
                        long e[4];
                        unit(d, e);
                        const long Pm[4] = {P[0] - e[0], P[1] - e[1], P[2] - e[2], P[3] - e[3]};
                        const long Pp[4] = {P[0] + e[0], P[1] + e[1], P[2] + e[2], P[3] + e[3]};
                        double gm[4], gp[4];
                        face_gradient(get_padded, &ctx, h, d, Pm, gm); /* -e_d face of P */
                        face_gradient(get_padded, &ctx, h, d, P, gp);  /* +e_d face of P */
                        q[2 * d] = gm[0] * gm[0] + gm[1] * gm[1] + gm[2] * gm[2] + gm[3] * gm[3];
                        q[2 * d + 1] = gp[0] * gp[0] + gp[1] * gp[1] + gp[2] * gp[2] + gp[3] * gp[3];
                        Gf[2 * d] = G[(size_t)d * np + pidx(n, Pm[0], Pm[1], Pm[2], Pm[3])];
                        Gf[2 * d + 1] = G[(size_t)d * np + pidx(n, P[0], P[1], P[2], P[3])];
                        for (int t = 0; t < 4; ++t) { nb[2 * d][t] = Pm[t]; nb[2 * d + 1][t] = Pp[t]; }
                    }
                    double qs = 0.0;
                    for (int f = 0; f < 8; ++f) qs += q[f];
                    const double Abar = sqrt(eps * eps + qs / 8.0);
                    const size_t c = iidx(n, i, j, k, l);
                    double rhs = w[pidx(n, i, j, k, l)];
                    for (int f = 0; f < 8; ++f) {
                        const double A = sqrt(eps * eps + q[f]);
                        const double cf = th2 * Abar * Gf[f] / A;
                        coef[c * 8 + f] = cf;
                        const int d = f / 2;
                        if (nb[f][d] < 1 || nb[f][d] > n[d]) /* ghost neighbour */
                            rhs += cf * ub[pidx(n, nb[f][0], nb[f][1], nb[f][2], nb[f][3])];
                    }
                    b[c] = rhs;
                }
}

/* ------------------------------------------------------------------ SOR */

static double diag_of(const double *cf)
{
    double s = 1.0;
    for (int f = 0; f < 8; ++f) s += cf[f];
    return s;
}

/* b_P + sum over interior neighbours of c_f * u_nbr  (ghost terms are in b) */
static double off_sum(const int *n, const double *coef, const double *b, const double *u, long i,
                      long j, long k, long l)
{
    const size_t c = iidx(n, i, j, k, l);
    const double *cf = coef + c * 8;
    const long P[4] = {i, j, k, l};
    double s = b[c];
    for (int f = 0; f < 8; ++f) {
        const int d = f / 2;
        long q[4] = {P[0], P[1], P[2], P[3]};
        q[d] += (f & 1) ? 1 : -1;
        if (q[d] < 1 || q[d] > n[d]) continue;
        s += cf[f] * u[pidx(n, q[0], q[1], q[2], q[3])];
    }
    return s;
}

/* ||b - A u||_2^2 over interior rows, summed frame by frame in a fixed order */
static double residual2(const int *n, const double *coef, const double *b, const double *u)
{
    double *part = (double *)calloc((size_t)n[3], sizeof(double));
#pragma omp parallel for schedule(static)
    for (long l = 1; l <= n[3]; ++l) {
        double acc = 0.0;
        for (long k = 1; k <= n[2]; ++k)
            for (long j = 1; j <= n[1]; ++j)
                for (long i = 1; i <= n[0]; ++i) {
                    const size_t c = iidx(n, i, j, k, l);
                    const double r = off_sum(n, coef, b, u, i, j, k, l) - diag_of(coef + c * 8) * u[pidx(n, i, j, k, l)];
                    acc += r * r;
                }
        part[l - 1] = acc;
    }
    double tot = 0.0;
    for (long l = 0; l < n[3]; ++l) tot += part[l];
    free(part);
    return tot;
}

static void sor_update(const int *n, const double *coef, const double *b, double *u, double omega,
                       long i, long j, long k, long l)
{
    const size_t c = iidx(n, i, j, k, l);
    const double ubar = off_sum(n, coef, b, u, i, j, k, l) / diag_of(coef + c * 8);
    const size_t p = pidx(n, i, j, k, l);
    u[p] = omega * ubar + (1.0 - omega) * u[p];
}

/*
 * SOR for the step system (Sec. 3.2.2: the SOR relaxation of a Gauss-Seidel
 * value, and its red-black variant).
 *   order 0: lexicographic, loops l -> k -> j -> i (i innermost), in place, so
 *            the -e_d neighbours already hold new values;
 *   order 1: red-black: all cells with (i+j+k+l) even, then all odd ones.
 * Stopping rule (the paper only says a residual criterion is checked):
 *   R_k = ||b - A u^(k)||_2 over interior rows; check k=0, then after every
 *   check_every-th iteration; stop at the first R_k <= tol*||b||_2 and return
 *   u^(k).  u: padded, in = initial guess, out = result (ghosts untouched).
 * Returns 0 when converged, 1 when max_iter was reached.
 * Pinned: dense LU on small grids; lexicographic and red-black reach the same
 * fixed point.
 */
int oracle_sor(const int *n, int order, double omega, double tol, int max_iter, int check_every,
               const double *coef, const double *b, double *u, int *iterations, double *rel_res)
{
    const double bn = norm2_interior(n, b);
    double R = sqrt(residual2(n, coef, b, u));
    *iterations = 0;
    *rel_res = bn > 0.0 ? R / bn : R;
    if (R <= tol * bn) return 0;
    if (check_every < 1) check_every = 1;
    for (int it = 1; it <= max_iter; ++it) {
        if (order == 0) {
            for (long l = 1; l <= n[3]; ++l)
                for (long k = 1; k <= n[2]; ++k)
                    for (long j = 1; j <= n[1]; ++j)
                        for (long i = 1; i <= n[0]; ++i) sor_update(n, coef, b, u, omega, i, j, k, l);
        } else {
            for (int colour = 0; colour < 2; ++colour) {
#pragma omp parallel for schedule(static)
                for (long l = 1; l <= n[3]; ++l)
                    for (long k = 1; k <= n[2]; ++k)
                        for (long j = 1; j <= n[1]; ++j)
                            for (long i = 1; i <= n[0]; ++i)
                                if (((i + j + k + l) & 1) == colour) sor_update(n, coef, b, u, omega, i, j, k, l);
            }
        }
        *iterations = it;
        if (it % check_every == 0 || it == max_iter) {
            R = sqrt(residual2(n, coef, b, u));
            *rel_res = bn > 0.0 ? R / bn : R;
            if (R <= tol * bn) return 0;
        }
    }
    return 1;
}

/* ----------------------------------------------------------- rescaling */

/*
 * Local rescaling (Sec. 3.2.2, local rescaling remark): for each frame and
 * ball, mu = min and xi = max of u over the ball (all computed from the input
 * u before any cell changes); every cell owned by the ball (owner map) becomes
 * (u - mu) / (xi - mu).  A ball with xi - mu < 1e-12 is left unchanged (reading:
 * the division is undefined there).  Cells in no ball and ghosts are unchanged.
 * u: padded.
 */
void oracle_rescale(const int *n, const oracle_centre *cs, int nc, double r, const int32_t *owner,
                    double *u)
{
    const size_t ni = (size_t)n[0] * n[1] * n[2] * n[3];
    double *ui = (double *)malloc(ni * sizeof(double));
    for (long l = 1; l <= n[3]; ++l)
        for (long k = 1; k <= n[2]; ++k)
            for (long j = 1; j <= n[1]; ++j)
                for (long i = 1; i <= n[0]; ++i) ui[iidx(n, i, j, k, l)] = u[pidx(n, i, j, k, l)];
    double *mu = (double *)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(double));
    double *xi = (double *)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(double));
    ball_minmax_interior(n, cs, nc, r, ui, mu, xi);
    for (long l = 1; l <= n[3]; ++l)
        for (long k = 1; k <= n[2]; ++k)
            for (long j = 1; j <= n[1]; ++j)
                for (long i = 1; i <= n[0]; ++i) {
                    const int m = owner[iidx(n, i, j, k, l)];
                    if (m < 0) continue;
                    if (!(xi[m] - mu[m] >= 1e-12)) continue;
                    const size_t p = pidx(n, i, j, k, l);
                    u[p] = (u[p] - mu[m]) / (xi[m] - mu[m]);
                }
    free(ui);
    free(mu);
    free(xi);
}

/* number of OpenMP threads the red-black loops use (1 without OpenMP) */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------ cell tracking */

/*
 * Cell tracking from the 4D segmentation (Sec. 5, "Cell tracking based on 4D
 * segmentation").  Readings where the section is silent:
 *  - a voxel of frame l is segmented when u >= level (u after the last step;
 *    the level is a parameter, 0.5 for rescaled u in [0,1]);
 *  - a "segmented cell" is a set of segmented voxels of one frame connected
 *    through shared faces (6-neighbourhood); it is named by the smallest
 *    interior index of its voxels (a name unique over all frames);
 *  - "distance from the segmented cell boundary" is the Euclidean distance to
 *    the nearest voxel of the same frame outside the cell, the region outside
 *    the image counting as outside; the centre is the voxel where it is
 *    largest, ties to the smallest index.
 *
 * Labels (interior int32): the cell name, -1 for voxels outside every cell.
 * Flood fill from every unlabelled segmented voxel in increasing index order,
 * so the first voxel reached is the smallest of its cell.
 */
void oracle_track_label(const int *n, const double *u, double level, int32_t *label)
{
    const size_t ni = (size_t)n[0] * n[1] * n[2] * n[3];
    long *queue = (long *)malloc(ni * sizeof(long) * 4 + 4 * sizeof(long));
    for (size_t q = 0; q < ni; ++q) label[q] = -1;
    for (long l = 1; l <= n[3]; ++l)
        for (long k = 1; k <= n[2]; ++k)
            for (long j = 1; j <= n[1]; ++j)
                for (long i = 1; i <= n[0]; ++i) {
                    const size_t q0 = iidx(n, i, j, k, l);
                    if (label[q0] >= 0 || !(u[pidx(n, i, j, k, l)] >= level)) continue;
                    const int32_t name = (int32_t)q0;
                    size_t head = 0, tail = 0;
                    label[q0] = name;
                    queue[tail++] = i; queue[tail++] = j; queue[tail++] = k;
                    while (head < tail) {
                        const long ci = queue[head], cj = queue[head + 1], ck = queue[head + 2];
                        head += 3;
                        const long nb[6][3] = {{ci - 1, cj, ck}, {ci + 1, cj, ck}, {ci, cj - 1, ck},
                                               {ci, cj + 1, ck}, {ci, cj, ck - 1}, {ci, cj, ck + 1}};
                        for (int s = 0; s < 6; ++s) {
                            const long a = nb[s][0], b = nb[s][1], c = nb[s][2];
                            if (a < 1 || a > n[0] || b < 1 || b > n[1] || c < 1 || c > n[2]) continue;
                            const size_t qn = iidx(n, a, b, c, l);
                            if (label[qn] >= 0 || !(u[pidx(n, a, b, c, l)] >= level)) continue;
                            label[qn] = name;
                            queue[tail++] = a; queue[tail++] = b; queue[tail++] = c;
                        }
                    }
                }
    free(queue);
}

/*
 * Squared distance (voxel units) of every voxel of a cell to the nearest voxel
 * of its frame outside the cell, by brute force over the frame and its
 * one-voxel outer shell (outside the image); 0 for voxels in no cell.
 * O(cells' voxels x frame voxels): small grids only.
 */
void oracle_track_dist2(const int *n, const int32_t *label, int32_t *d2)
{
    const size_t ni = (size_t)n[0] * n[1] * n[2] * n[3];
    for (size_t q = 0; q < ni; ++q) d2[q] = 0;
#pragma omp parallel for schedule(dynamic)
    for (long l = 1; l <= n[3]; ++l)
        for (long k = 1; k <= n[2]; ++k)
            for (long j = 1; j <= n[1]; ++j)
                for (long i = 1; i <= n[0]; ++i) {
                    const size_t q = iidx(n, i, j, k, l);
                    const int32_t own = label[q];
                    if (own < 0) continue;
                    long best = -1;
                    for (long c = 0; c <= n[2] + 1; ++c)
                        for (long b = 0; b <= n[1] + 1; ++b)
                            for (long a = 0; a <= n[0] + 1; ++a) {
                                const int outside = a < 1 || a > n[0] || b < 1 || b > n[1] || c < 1 || c > n[2];
                                if (!outside && label[iidx(n, a, b, c, l)] == own) continue;
                                const long dd = (a - i) * (a - i) + (b - j) * (b - j) + (c - k) * (c - k);
                                if (best < 0 || dd < best) best = dd;
                            }
                    d2[q] = (int32_t)best;
                }
}

/*
 * One record per cell, in increasing name order: name, frame, centre (interior
 * index of the voxel of largest d2, ties to the smallest index), its d2, and
 * the link to the previous frame by the backtracking of Sec. 5: the cell of
 * frame l-1 that contains the centre's voxel moved to frame l-1 (kind 1);
 * otherwise the cell of frame l-1 that overlaps most voxels of this cell moved
 * to frame l-1, ties to the smallest name (kind 2); otherwise none (-1, kind 0).
 * rec: capacity x 6 int32 (name, frame, centre, d2, prev, kind).  Returns the
 * number of cells, or -1 if it exceeds the capacity.
 */
int oracle_track_cells(const int *n, const int32_t *label, const int32_t *d2, int32_t *rec, int capacity)
{
    const size_t ni = (size_t)n[0] * n[1] * n[2] * n[3];
    const size_t fsz = (size_t)n[0] * n[1] * n[2];
    int32_t *slot = (int32_t *)malloc(ni * sizeof(int32_t));     /* record of the cell a name names */
    int nc = 0;
    for (size_t q = 0; q < ni; ++q) {
        slot[q] = -1;
        if (label[q] != (int32_t)q) continue;          /* q names its cell */
        if (nc >= capacity) { free(slot); return -1; }
        int32_t *r = rec + 6 * nc;
        r[0] = (int32_t)q;
        r[1] = (int32_t)(q / fsz);
        r[2] = (int32_t)q;
        r[3] = d2[q];
        r[4] = -1;
        r[5] = 0;
        slot[q] = nc;
        ++nc;
    }
    /* centres: scan voxels in increasing index; strict '>' keeps the smallest */
    for (size_t q = 0; q < ni; ++q) {
        if (label[q] < 0) continue;
        int32_t *r = rec + 6 * slot[label[q]];
        if (d2[q] > r[3]) { r[3] = d2[q]; r[2] = (int32_t)q; }
    }
    int32_t *cand = (int32_t *)malloc(fsz * sizeof(int32_t));
    long *count = (long *)malloc(fsz * sizeof(long));
    for (int c = 0; c < nc; ++c) {
        int32_t *r = rec + 6 * c;
        if (r[1] == 0) continue;
        const int32_t below = label[(size_t)r[2] - fsz];
        if (below >= 0) { r[4] = below; r[5] = 1; continue; }
        /* overlap counts with the cells of the previous frame: a list of
         * (candidate, count) pairs over this cell's voxels */
        int nk = 0;
        for (size_t q = (size_t)r[1] * fsz; q < (size_t)(r[1] + 1) * fsz; ++q) {
            if (label[q] != r[0]) continue;
            const int32_t b = label[q - fsz];
            if (b < 0) continue;
            int t = 0;
            while (t < nk && cand[t] != b) ++t;
            if (t == nk) { cand[nk] = b; count[nk] = 0; ++nk; }
            ++count[t];
        }
        int32_t best = -1;
        long best_count = 0;
        for (int t = 0; t < nk; ++t)
            if (count[t] > best_count || (count[t] == best_count && cand[t] < best)) {
                best = cand[t];
                best_count = count[t];
            }
        if (best >= 0) { r[4] = best; r[5] = 2; }
    }
    free(cand);
    free(count);
    free(slot);
    return nc;
}
