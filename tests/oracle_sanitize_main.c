/*
 * Test harness: runs every oracle routine on small seeded inputs (odd, even
 * and unit extents, balls crossing the box, the lexicographic and the
 * red-black solve, Dirichlet data in the ghosts) so that a build with the
 * address and undefined-behaviour sanitizers can check the oracle's memory
 * accesses and arithmetic.  Compiled together with oracle/subsurf4d_oracle.c
 * by tests/test_oracle_sanitizers.py; exits 0 when every call returned.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    float x, y, z;
    int32_t frame;
} centre;

void oracle_owner_map(const int *n, const centre *cs, int nc, double r, int32_t *owner);
void oracle_threshold(const int *n, const double *I0, const centre *cs, int nc, double r, double lam,
                      const int32_t *owner, double *out);
int oracle_lhe_step(const int *n, double h, double tau_s, double omega, double tol, int max_iter,
                    const double *J, double *out);
void oracle_face_gradient(const int *n, double h, const double *v, int d, double *out);
void oracle_face_g(const int *n, double h, double K, double delta, double vartheta, const double *a,
                   const double *b, double *G);
void oracle_init_u(const int *n, const centre *cs, int nc, double v, double R, double *u);
void oracle_assemble(const int *n, double h, double eps, double tau, const double *G, const double *w,
                     const double *ub, double *coef, double *b);
int oracle_sor(const int *n, int order, double omega, double tol, int max_iter, int check_every,
               const double *coef, const double *b, double *u, int *iterations, double *rel_res);
void oracle_rescale(const int *n, const centre *cs, int nc, double r, const int32_t *owner, double *u);

static uint64_t state = 88172645463325252ull;
static double rnd(void)
{
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (double)(state >> 11) / 9007199254740992.0;
}

static int run(const int n[4])
{
    const size_t ni = (size_t)n[0] * n[1] * n[2] * n[3];
    const size_t np = (size_t)(n[0] + 2) * (n[1] + 2) * (n[2] + 2) * (n[3] + 2);
    double *I0 = malloc(ni * sizeof(double)), *ITH = malloc(ni * sizeof(double));
    double *S0 = malloc(ni * sizeof(double)), *S1 = malloc(ni * sizeof(double));
    double *G = malloc(4 * np * sizeof(double)), *grad = malloc(4 * np * sizeof(double));
    double *u = malloc(np * sizeof(double)), *ub = malloc(np * sizeof(double));
    double *coef = malloc(8 * ni * sizeof(double)), *b = malloc(ni * sizeof(double));
    int32_t *owner = malloc(ni * sizeof(int32_t));
    centre cs[6];
    const int nc = 6;
    for (int m = 0; m < nc; ++m) {
        cs[m].x = (float)(rnd() * (n[0] + 4) - 2);
        cs[m].y = (float)(rnd() * (n[1] + 4) - 2);
        cs[m].z = (float)(rnd() * (n[2] + 4) - 2);
        cs[m].frame = (int32_t)(rnd() * (n[3] + 2)) - 1;   /* some outside the frames */
    }
    for (size_t q = 0; q < ni; ++q) I0[q] = rnd();
    for (size_t q = 0; q < np; ++q) ub[q] = rnd();
    oracle_owner_map(n, cs, nc, 2.5, owner);
    oracle_threshold(n, I0, cs, nc, 2.5, 0.5, owner, ITH);
    if (oracle_lhe_step(n, 1.0, 0.1, 1.3, 1e-12, 10000, I0, S0) < 0) return 1;
    if (oracle_lhe_step(n, 1.0, 0.1, 1.3, 1e-12, 10000, ITH, S1) < 0) return 1;
    for (int d = 0; d < 4; ++d) oracle_face_gradient(n, 1.0, ub, d, grad);
    oracle_face_g(n, 1.0, 1000.0, 0.5, 0.5, S0, S1, G);
    oracle_init_u(n, cs, nc, 1.0, 0.0, u);
    oracle_init_u(n, cs, nc, 1.0, 3.0, u);
    oracle_rescale(n, cs, nc, 2.5, owner, u);
    for (int order = 0; order < 2; ++order) {
        int it = 0;
        double rr = 0.0;
        oracle_assemble(n, 1.0, 1e-3, 0.5, G, u, ub, coef, b);
        oracle_sor(n, order, 1.5, 1e-10, 5000, order ? 2 : 1, coef, b, u, &it, &rr);
        if (!(rr == rr)) return 2;
        oracle_rescale(n, cs, nc, 2.5, owner, u);
    }
    free(I0); free(ITH); free(S0); free(S1); free(G); free(grad); free(u); free(ub); free(coef); free(b);
    free(owner);
    return 0;
}

int main(void)
{
    const int shapes[][4] = {{1, 1, 1, 1}, {2, 1, 1, 1}, {5, 4, 3, 3}, {6, 7, 2, 4}, {9, 3, 4, 2}};
    for (size_t s = 0; s < sizeof(shapes) / sizeof(shapes[0]); ++s) {
        const int rc = run(shapes[s]);
        if (rc) {
            fprintf(stderr, "shape %zu failed: %d\n", s, rc);
            return rc;
        }
    }
    printf("oracle sanitizer run ok\n");
    return 0;
}
