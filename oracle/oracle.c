/*
 * oracle.c -- plain, slow FP64 CPU reference for the tetrahedral FMM.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no source with the HIP path.
 *
 * What it computes (Palmesi et al., "Highly Parallel Demagnetization Field
 * Calculation Using the Fast Multipole Method on Tetrahedral Meshes with
 * Continuous Sources"):
 *
 *   u(x) = 1/(4 pi) sum_T  int_T  M_T(r') . grad' (1/|x - r'|) dr'     (eq. approx1)
 *
 * with M_T affine on each tetrahedron (nodal values, barycentric interpolation).
 *
 *   orc_tet_potential   exact potential of one linearly magnetised tetrahedron
 *                       (Sec. 2.1; evaluated by integration by parts into face
 *                       single-layer potentials, Wilton et al. 1984 closed forms)
 *   orc_direct          O(N^2) sum of orc_tet_potential over all tets
 *   orc_fmm_*           the FMM of Secs. 2-3: octree (Sec. 3.1), MAC (Sec. 3.2),
 *                       dual tree traversal (Sec. 3.3, Listings 1-2), P2M by an
 *                       exact simplex quadrature (eq. expCoeffs), M2M, M2L, L2L,
 *                       L2P of the Cartesian Taylor expansion (Secs. 2.2-2.3)
 *
 * Readings of the paper that this file fixes (all listed in the design notes):
 *  - order p means |n| <= p; M2L truncates at |n|+|m| <= p; Q_0 = 0.
 *  - expansion centres are the geometric centres of the octree cubes.
 *  - MAC: r_tgt(A) + r_src(B) < theta |c_A - c_B|, strict, compared squared.
 *  - traversal: MAC first, then both-leaf -> P2P, else split the cell with the
 *    larger side (ties split the source; a leaf is never split).
 *  - a cell is split while it holds more than `leaf` tets or targets.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (see build.py).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846
#define ORC_INV4PI (0.25 / ORC_PI)
#define ORC_MAXP 12
#define ORC_MAXDEPTH 21

/* ------------------------------------------------------------------------- */
/* small vector helpers                                                       */
/* ------------------------------------------------------------------------- */
static double dot3(const double *a, const double *b) { return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]; }
static void sub3(const double *a, const double *b, double *r) { r[0] = a[0] - b[0]; r[1] = a[1] - b[1]; r[2] = a[2] - b[2]; }
static void cross3(const double *a, const double *b, double *r)
{
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}
static double norm3(const double *a) { return sqrt(dot3(a, a)); }

/* ------------------------------------------------------------------------- */
/* Single-layer potentials of a flat triangle (Wilton et al., IEEE TAP 1984). */
/*                                                                            */
/*   I0    = int_F 1/|x-y| dA                                                 */
/*   I1[3] = int_F (y - rho)/|x-y| dA,  rho = projection of x on the plane    */
/*                                                                            */
/* p[0..2] are the corners, counter-clockwise seen from the side n points to. */
/* Per edge: t0 signed in-plane distance of rho to the edge line (positive    */
/* on the inner side), l+/l- the coordinates of the edge ends along the edge, */
/* R0 the distance of x to the edge line, R+/R- the distances to the ends.    */
/* ------------------------------------------------------------------------- */
static void orc_triangle_potentials(const double *x, const double *p[3], const double *n, double *I0, double I1[3])
{
    double xp[3], rho[3];
    sub3(x, p[0], xp);
    double w = dot3(n, xp); /* height of x above the face plane */
    for (int j = 0; j < 3; ++j) /* x at a corner lies in the plane exactly */
        if (x[0] == p[j][0] && x[1] == p[j][1] && x[2] == p[j][2]) w = 0.0;
    for (int d = 0; d < 3; ++d) rho[d] = x[d] - w * n[d];
    double aw = fabs(w);
    double s0 = 0.0, s1[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 3; ++i) {
        const double *rm = p[i], *rp = p[(i + 1) % 3];
        double e[3], lhat[3], uhat[3], dm[3], dp[3];
        sub3(rp, rm, e);
        double len = norm3(e);
        for (int d = 0; d < 3; ++d) lhat[d] = e[d] / len;
        cross3(lhat, n, uhat); /* outward in-plane normal of the edge */
        sub3(rm, rho, dm);
        sub3(rp, rho, dp);
        double t0 = dot3(dm, uhat);
        double lm = dot3(dm, lhat), lp = dot3(dp, lhat);
        double R0sq = t0 * t0 + w * w;
        double xm[3], xpp[3];
        sub3(x, rm, xm);
        sub3(x, rp, xpp);
        double Rm = norm3(xm), Rp = norm3(xpp);
        if (R0sq > 0.0 && Rm > 0.0 && Rp > 0.0) {
            /* f = ln((R+ + l+)/(R- + l-)), in the form free of cancellation;
               its factors t0 and R0^2 vanish when x is on the edge line */
            double f;
            if (lm >= 0.0)
                f = log((Rp + lp) / (Rm + lm));
            else if (lp <= 0.0)
                f = log((Rm - lm) / (Rp - lp));
            else
                f = log((Rp + lp) * (Rm - lm) / R0sq);
            s0 += t0 * f;
            for (int d = 0; d < 3; ++d) s1[d] += 0.5 * uhat[d] * (R0sq * f);
        }
        for (int d = 0; d < 3; ++d) s1[d] += 0.5 * uhat[d] * (lp * Rp - lm * Rm);
        if (aw > 0.0 && t0 != 0.0)
            s0 -= aw * (atan(t0 * lp / (R0sq + aw * Rp)) - atan(t0 * lm / (R0sq + aw * Rm)));
    }
    *I0 = s0;
    I1[0] = s1[0];
    I1[1] = s1[1];
    I1[2] = s1[2];
}

/* ------------------------------------------------------------------------- */
/* Potential at x of one tetrahedron with affine magnetisation (eq. approx1,  */
/* one term).  v[4][3] corners (either orientation), M[4][3] nodal values.    */
/*                                                                            */
/* Integration by parts:                                                      */
/*   int_T M.grad'(1/|x-r'|) = sum_faces int_F (M.n)/|x-y| dA                 */
/*                             - div M int_T 1/|x-r'| dr'                     */
/* and int_T 1/|x-r'| = 1/2 sum_faces h_F int_F 1/|x-y| dA, h_F = n.(y-x).    */
/* M.n is affine on a face:  M(y).n = M(rho).n + (G^T n).(y - rho),           */
/* G = dM/dy (constant), so each face needs I0 and I1 only.                   */
/* ------------------------------------------------------------------------- */
double orc_tet_potential(const double *x, const double *v, const double *M)
{
    const double *V[4] = {v, v + 3, v + 6, v + 9};
    double e1[3], e2[3], e3[3], c23[3], c31[3], c12[3];
    sub3(V[1], V[0], e1);
    sub3(V[2], V[0], e2);
    sub3(V[3], V[0], e3);
    cross3(e2, e3, c23);
    cross3(e3, e1, c31);
    cross3(e1, e2, c12);
    double det = dot3(e1, c23);
    /* gradients of barycentric coordinates: rows of the inverse Jacobian */
    double g[4][3];
    for (int d = 0; d < 3; ++d) {
        g[1][d] = c23[d] / det;
        g[2][d] = c31[d] / det;
        g[3][d] = c12[d] / det;
        g[0][d] = -(g[1][d] + g[2][d] + g[3][d]);
    }
    /* G[a][b] = dM_a/dy_b */
    double G[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int i = 0; i < 4; ++i) s += M[3 * i + a] * g[i][b];
            G[a][b] = s;
        }
    double divM = G[0][0] + G[1][1] + G[2][2];
    /* M at x by the affine extension */
    double lam[4], xv[3];
    sub3(x, V[0], xv);
    lam[1] = dot3(g[1], xv);
    lam[2] = dot3(g[2], xv);
    lam[3] = dot3(g[3], xv);
    lam[0] = 1.0 - (lam[1] + lam[2] + lam[3]);
    double Mx[3];
    for (int a = 0; a < 3; ++a) {
        double s = 0.0;
        for (int i = 0; i < 4; ++i) s += lam[i] * M[3 * i + a];
        Mx[a] = s;
    }

    double total = 0.0;
    for (int k = 0; k < 4; ++k) {
        /* face opposite corner k */
        const double *p[3];
        int j = 0;
        for (int i = 0; i < 4; ++i)
            if (i != k) p[j++] = V[i];
        double a1[3], a2[3], nn[3];
        sub3(p[1], p[0], a1);
        sub3(p[2], p[0], a2);
        cross3(a1, a2, nn);
        double nl = norm3(nn);
        double n[3] = {nn[0] / nl, nn[1] / nl, nn[2] / nl};
        double tok[3];
        sub3(V[k], p[0], tok);
        if (dot3(n, tok) > 0.0) { /* make n point away from the tetrahedron */
            n[0] = -n[0];
            n[1] = -n[1];
            n[2] = -n[2];
            const double *t = p[1];
            p[1] = p[2];
            p[2] = t;
        }
        double I0, I1[3];
        orc_triangle_potentials(x, p, n, &I0, I1);
        double yx[3];
        sub3(p[0], x, yx);
        double h = dot3(n, yx);
        double Gn[3], GTn[3];
        for (int a = 0; a < 3; ++a) {
            Gn[a] = G[a][0] * n[0] + G[a][1] * n[1] + G[a][2] * n[2];
            GTn[a] = G[0][a] * n[0] + G[1][a] * n[1] + G[2][a] * n[2];
        }
        double sigma_rho = dot3(Mx, n) + h * dot3(n, Gn); /* M(rho).n */
        total += sigma_rho * I0 + dot3(GTn, I1) - 0.5 * divM * h * I0;
    }
    return ORC_INV4PI * total;
}

/* ------------------------------------------------------------------------- */
/* Far pairs.  The closed forms above add face and edge terms that are each  */
/* larger than their sum by about (d/diam)^2 to (d/diam)^3 (d the distance   */
/* of x from the tet, diam its longest edge), so far from the tet they lose  */
/* that many digits to cancellation.  There the integrand of eq. approx1 is  */
/* smooth on the tet and a Gauss product rule is accurate instead:           */
/*                                                                            */
/*   u_T(x) = 1/(4 pi) int_T M(r') . (x - r') / |x - r'|^3 dr'                */
/*                                                                            */
/* on the collapsed cube: lambda1 = a, lambda2 = b (1 - a),                   */
/* lambda3 = c (1 - a)(1 - b), dr' = 6 |V| (1 - a)^2 (1 - b) da db dc, with   */
/* n-point Gauss-Legendre in a, b and c.  A polynomial of total degree q in  */
/* r' becomes one of degree q + 2, q + 1, q in a, b, c, so the rule is exact */
/* to total degree 2n - 3 (13 for n = 8).                                     */
/* ------------------------------------------------------------------------- */
#define ORC_GL_MAX 24

/* n-point Gauss-Legendre nodes and weights on [0, 1] (Newton on P_n from the */
/* usual cosine guesses; P_n and P_n' by the three-term recurrence).          */
static void orc_gauss_legendre01(int n, double *t, double *w)
{
    for (int i = 0; i < n; ++i) {
        double x = cos(ORC_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
            const double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) <= 1e-16) break; /* quadratic convergence: one step past this is round-off */
        }
        /* recompute P_n' at the converged node for the weight */
        {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
        }
        t[i] = 0.5 * (1.0 - x);
        w[i] = 1.0 / ((1.0 - x * x) * dp * dp); /* half the [-1, 1] weight 2/((1-x^2) P_n'^2) */
    }
}

/* The 1-D rule, exported for its pin. */
int orc_gauss_legendre01_rule(int n, double *t, double *w)
{
    if (n < 1 || n > ORC_GL_MAX) return -1;
    orc_gauss_legendre01(n, t, w);
    return 0;
}

/* u_T(x) by the n^3-point product rule built on the 1-D rule (t, w). */
static double orc_tet_potential_gauss_rule(const double *x, const double *v, const double *M, int n, const double *t,
                                           const double *w)
{
    double e1[3], e2[3], e3[3], c23[3];
    sub3(v + 3, v, e1);
    sub3(v + 6, v, e2);
    sub3(v + 9, v, e3);
    cross3(e2, e3, c23);
    const double vol6 = fabs(dot3(e1, c23));
    double total = 0.0;
    for (int ia = 0; ia < n; ++ia)
        for (int ib = 0; ib < n; ++ib)
            for (int ic = 0; ic < n; ++ic) {
                const double a = t[ia], b = t[ib], c = t[ic];
                const double l1 = a, l2 = b * (1.0 - a), l3 = c * (1.0 - a) * (1.0 - b);
                const double l0 = 1.0 - l1 - l2 - l3;
                const double wt = w[ia] * w[ib] * w[ic] * (1.0 - a) * (1.0 - a) * (1.0 - b);
                double y[3], m[3], d[3];
                for (int k = 0; k < 3; ++k) {
                    y[k] = v[k] + l1 * e1[k] + l2 * e2[k] + l3 * e3[k];
                    m[k] = l0 * M[k] + l1 * M[3 + k] + l2 * M[6 + k] + l3 * M[9 + k];
                    d[k] = x[k] - y[k];
                }
                const double r = norm3(d);
                total += wt * dot3(m, d) / (r * r * r);
            }
    return ORC_INV4PI * vol6 * total;
}

double orc_tet_potential_gauss(const double *x, const double *v, const double *M, int n)
{
    if (n < 1 || n > ORC_GL_MAX) return NAN;
    double t[ORC_GL_MAX], w[ORC_GL_MAX];
    orc_gauss_legendre01(n, t, w);
    return orc_tet_potential_gauss_rule(x, v, M, n, t, w);
}

/* Distance of x from the centroid of the tet in units of its longest edge. */
double orc_tet_distance_ratio(const double *x, const double *v)
{
    double c[3], d[3], diam = 0.0;
    for (int k = 0; k < 3; ++k) c[k] = ((v[k] + v[3 + k]) + (v[6 + k] + v[9 + k])) * 0.25;
    for (int a = 0; a < 4; ++a)
        for (int b = a + 1; b < 4; ++b) {
            sub3(v + 3 * b, v + 3 * a, d);
            const double l = norm3(d);
            if (l > diam) diam = l;
        }
    sub3(x, c, d);
    return norm3(d) / diam;
}

/* The pair as the direct sum takes it: the closed form within 3 diameters,  */
/* the 8-point (degree 13) Gauss product rule beyond.  Measured on random    */
/* tets (error relative to |M| V / (4 pi d^2)): the closed form loses about  */
/* (d/diam)^4 eps, ~1e-12 at 3 diameters, up to 1e-10 at 4 and ~1e-9 at 10,  */
/* while the rule is at ~1e-13 from 2 diameters and at round-off from 3.     */
#define ORC_FAR_RATIO 3.0
#define ORC_FAR_POINTS 8
static double orc_pair_direct(const double *x, const double *v, const double *M, const double *t, const double *w)
{
    if (orc_tet_distance_ratio(x, v) >= ORC_FAR_RATIO) return orc_tet_potential_gauss_rule(x, v, M, ORC_FAR_POINTS, t, w);
    return orc_tet_potential(x, v, M);
}

double orc_tet_potential_direct(const double *x, const double *v, const double *M)
{
    double t[ORC_FAR_POINTS], w[ORC_FAR_POINTS];
    orc_gauss_legendre01(ORC_FAR_POINTS, t, w);
    return orc_pair_direct(x, v, M, t, w);
}

/* ------------------------------------------------------------------------- */
/* O(N^2) direct sum: u[f][i] = sum_T u_T(target_i) for field f, every pair  */
/* by orc_tet_potential_direct.                                               */
/* nodes [n_nodes][3], tets [n_tets][4] (0-based), M [F][n_nodes][3],         */
/* targets [n_targets][3], u [F][n_targets].  Returns 0 or -1 on bad input.   */
/* ------------------------------------------------------------------------- */
int orc_direct(const double *nodes, int64_t n_nodes, const int32_t *tets, int64_t n_tets, const double *M, int32_t F,
               const double *targets, int64_t n_targets, double *u)
{
    for (int64_t t = 0; t < 4 * n_tets; ++t)
        if (tets[t] < 0 || tets[t] >= n_nodes) return -1;
    double gt[ORC_FAR_POINTS], gw[ORC_FAR_POINTS];
    orc_gauss_legendre01(ORC_FAR_POINTS, gt, gw);
    for (int32_t f = 0; f < F; ++f) {
        const double *Mf = M + (size_t)f * n_nodes * 3;
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t i = 0; i < n_targets; ++i) {
            double s = 0.0;
            for (int64_t t = 0; t < n_tets; ++t) {
                double v[12], m[12];
                for (int c = 0; c < 4; ++c) {
                    int32_t nd = tets[4 * t + c];
                    for (int d = 0; d < 3; ++d) {
                        v[3 * c + d] = nodes[3 * (size_t)nd + d];
                        m[3 * c + d] = Mf[3 * (size_t)nd + d];
                    }
                }
                s += orc_pair_direct(targets + 3 * i, v, m, gt, gw);
            }
            u[(size_t)f * n_targets + i] = s;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Multi-indices n = (nx,ny,nz), |n| <= p, graded: degree 0,1,..,p; inside a  */
/* degree, nx descending then ny descending.                                  */
/* ------------------------------------------------------------------------- */
typedef struct {
    int p, ncoef;
    int (*mi)[3];                                  /* [ncoef][3] */
    int idx[ORC_MAXP + 1][ORC_MAXP + 1][ORC_MAXP + 1]; /* -1 where |n| > p */
    double binom[2 * ORC_MAXP + 1][2 * ORC_MAXP + 1];
} orc_basis;

static void orc_basis_init(orc_basis *B, int p)
{
    B->p = p;
    B->ncoef = (p + 1) * (p + 2) * (p + 3) / 6;
    B->mi = malloc(sizeof(int[3]) * (size_t)B->ncoef);
    for (int a = 0; a <= ORC_MAXP; ++a)
        for (int b = 0; b <= ORC_MAXP; ++b)
            for (int c = 0; c <= ORC_MAXP; ++c) B->idx[a][b][c] = -1;
    int k = 0;
    for (int d = 0; d <= p; ++d)
        for (int nx = d; nx >= 0; --nx)
            for (int ny = d - nx; ny >= 0; --ny) {
                int nz = d - nx - ny;
                B->mi[k][0] = nx;
                B->mi[k][1] = ny;
                B->mi[k][2] = nz;
                B->idx[nx][ny][nz] = k++;
            }
    for (int n = 0; n <= 2 * ORC_MAXP; ++n)
        for (int r = 0; r <= 2 * ORC_MAXP; ++r) {
            if (r > n)
                B->binom[n][r] = 0.0;
            else if (r == 0 || r == n)
                B->binom[n][r] = 1.0;
            else
                B->binom[n][r] = B->binom[n - 1][r - 1] + B->binom[n - 1][r];
        }
}
static void orc_basis_free(orc_basis *B) { free(B->mi); }

/* y^n for all |n| <= p (graded order) */
static void orc_monomials(const orc_basis *B, const double *y, double *out)
{
    double pw[3][ORC_MAXP + 1];
    for (int d = 0; d < 3; ++d) {
        pw[d][0] = 1.0;
        for (int j = 1; j <= B->p; ++j) pw[d][j] = pw[d][j - 1] * y[d];
    }
    for (int k = 0; k < B->ncoef; ++k) out[k] = pw[0][B->mi[k][0]] * pw[1][B->mi[k][1]] * pw[2][B->mi[k][2]];
}

/* ------------------------------------------------------------------------- */
/* Taylor coefficients of the Coulomb kernel (Sec. 2.2):                      */
/*   1/|x - y| = sum_n a_n(x) y^n,  a_n(x) = (-1)^|n|/n! d^n/dx^n (1/|x|)     */
/* computed by the recurrence of Visscher & Apalkov (cited for the recursive  */
/* computation of the coefficients):                                          */
/*   |n| r^2 a_n = (2|n|-1) sum_i x_i a_{n-e_i} - (|n|-1) sum_i a_{n-2e_i}    */
/* ------------------------------------------------------------------------- */
static void orc_taylor(const orc_basis *B, const double *x, int pmax, double *a)
{
    double r2 = dot3(x, x);
    a[0] = 1.0 / sqrt(r2);
    for (int k = 1; k < B->ncoef; ++k) {
        const int *n = B->mi[k];
        int d = n[0] + n[1] + n[2];
        if (d > pmax) break;
        double s1 = 0.0, s2 = 0.0;
        for (int i = 0; i < 3; ++i) {
            if (n[i] >= 1) {
                int m[3] = {n[0], n[1], n[2]};
                m[i] -= 1;
                s1 += x[i] * a[B->idx[m[0]][m[1]][m[2]]];
            }
            if (n[i] >= 2) {
                int m[3] = {n[0], n[1], n[2]};
                m[i] -= 2;
                s2 += a[B->idx[m[0]][m[1]][m[2]]];
            }
        }
        a[k] = ((2.0 * d - 1.0) * s1 - (d - 1.0) * s2) / (d * r2);
    }
}

/* ------------------------------------------------------------------------- */
/* Exact integration over a tetrahedron: Grundmann-Moeller rule of degree     */
/* 2s+1 (Grundmann & Moeller 1978), barycentric points and weights for the    */
/* reference simplex of volume 1/6.                                           */
/* ------------------------------------------------------------------------- */
typedef struct {
    int npts;
    double (*lam)[4];
    double *w;
} orc_rule;

static double orc_fact(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

static void orc_rule_init(orc_rule *R, int s)
{
    const int n = 3, deg = 2 * s + 1;
    int cap = 0;
    for (int i = 0; i <= s; ++i) {
        int m = s - i; /* compositions of m into 4 parts */
        cap += (m + 3) * (m + 2) * (m + 1) / 6;
    }
    R->lam = malloc(sizeof(double[4]) * (size_t)cap);
    R->w = malloc(sizeof(double) * (size_t)cap);
    R->npts = 0;
    for (int i = 0; i <= s; ++i) {
        double den = (double)(deg + n - 2 * i);
        double wi = ((i % 2) ? -1.0 : 1.0) * pow(2.0, -2.0 * s) * pow(den, deg) / (orc_fact(i) * orc_fact(deg + n - i));
        int m = s - i;
        for (int b0 = 0; b0 <= m; ++b0)
            for (int b1 = 0; b1 <= m - b0; ++b1)
                for (int b2 = 0; b2 <= m - b0 - b1; ++b2) {
                    int b3 = m - b0 - b1 - b2;
                    double *L = R->lam[R->npts];
                    L[0] = (2.0 * b0 + 1.0) / den;
                    L[1] = (2.0 * b1 + 1.0) / den;
                    L[2] = (2.0 * b2 + 1.0) / den;
                    L[3] = (2.0 * b3 + 1.0) / den;
                    R->w[R->npts++] = wi;
                }
    }
}
static void orc_rule_free(orc_rule *R)
{
    free(R->lam);
    free(R->w);
}

/* ------------------------------------------------------------------------- */
/* P2M of one tet about c (eq. expCoeffs):                                    */
/*   Q_n = int_T M(r') . grad' (r'-c)^n dr' = sum_k n_k int_T M_k (r'-c)^{n-e_k}  */
/* The integrand has degree <= p, so a rule of degree >= p is exact.          */
/* Q is accumulated (+=).                                                     */
/* ------------------------------------------------------------------------- */
static void orc_p2m_tet_acc(const orc_basis *B, const orc_rule *R, const double *v, const double *M, const double *c, double *Q)
{
    double e1[3], e2[3], e3[3], cr[3];
    sub3(v + 3, v, e1);
    sub3(v + 6, v, e2);
    sub3(v + 9, v, e3);
    cross3(e2, e3, cr);
    double vol6 = fabs(dot3(e1, cr)); /* 6 |V| */
    double mono[(ORC_MAXP + 1) * (ORC_MAXP + 2) * (ORC_MAXP + 3) / 6];
    for (int q = 0; q < R->npts; ++q) {
        const double *L = R->lam[q];
        double y[3], Mq[3];
        for (int d = 0; d < 3; ++d) {
            y[d] = L[0] * v[d] + L[1] * v[3 + d] + L[2] * v[6 + d] + L[3] * v[9 + d] - c[d];
            Mq[d] = L[0] * M[d] + L[1] * M[3 + d] + L[2] * M[6 + d] + L[3] * M[9 + d];
        }
        orc_monomials(B, y, mono);
        double wq = R->w[q] * vol6;
        for (int k = 1; k < B->ncoef; ++k) {
            const int *n = B->mi[k];
            double s = 0.0;
            for (int i = 0; i < 3; ++i) {
                if (n[i] == 0) continue;
                int m[3] = {n[0], n[1], n[2]};
                m[i] -= 1;
                s += n[i] * Mq[i] * mono[B->idx[m[0]][m[1]][m[2]]];
            }
            Q[k] += wq * s;
        }
    }
}

/* M2M: Q_n(c_P) += sum_{k<=n} C(n,k) (c_C - c_P)^{n-k} Q_k(c_C) */
static void orc_m2m_acc(const orc_basis *B, const double *Qc, const double *delta, double *Qp)
{
    double dp[3][ORC_MAXP + 1];
    for (int d = 0; d < 3; ++d) {
        dp[d][0] = 1.0;
        for (int j = 1; j <= B->p; ++j) dp[d][j] = dp[d][j - 1] * delta[d];
    }
    for (int a = 0; a < B->ncoef; ++a) {
        const int *n = B->mi[a];
        double s = 0.0;
        for (int b = 0; b < B->ncoef; ++b) {
            const int *k = B->mi[b];
            if (k[0] > n[0] || k[1] > n[1] || k[2] > n[2]) continue;
            double c = B->binom[n[0]][k[0]] * B->binom[n[1]][k[1]] * B->binom[n[2]][k[2]];
            s += c * dp[0][n[0] - k[0]] * dp[1][n[1] - k[1]] * dp[2][n[2] - k[2]] * Qc[b];
        }
        Qp[a] += s;
    }
}

/* M2L: l_m(c_A) += 1/(4 pi) (-1)^|m| sum_{|n|>=1, |n|+|m|<=p} C(n+m,n) a_{n+m}(c_A - c_B) Q_n(c_B) */
/* (p = pt <= B->p: the order of the target cell's level)                   */
static void orc_m2l_acc_p(const orc_basis *B, const double *Qb, const double *R, double *La, int pt)
{
    double a[(ORC_MAXP + 1) * (ORC_MAXP + 2) * (ORC_MAXP + 3) / 6];
    orc_taylor(B, R, B->p, a);
    for (int im = 0; im < B->ncoef; ++im) {
        const int *m = B->mi[im];
        int dm = m[0] + m[1] + m[2];
        double s = 0.0;
        for (int in = 1; in < B->ncoef; ++in) {
            const int *n = B->mi[in];
            int dn = n[0] + n[1] + n[2];
            if (dn + dm > pt) break; /* graded order: all later n are of higher degree */
            double c = B->binom[n[0] + m[0]][n[0]] * B->binom[n[1] + m[1]][n[1]] * B->binom[n[2] + m[2]][n[2]];
            s += c * a[B->idx[n[0] + m[0]][n[1] + m[1]][n[2] + m[2]]] * Qb[in];
        }
        La[im] += ORC_INV4PI * ((dm % 2) ? -s : s);
    }
}
static void orc_m2l_acc(const orc_basis *B, const double *Qb, const double *R, double *La)
{
    orc_m2l_acc_p(B, Qb, R, La, B->p);
}

/* Zero the coefficients of degree above q (graded order: a tail). */
static void orc_truncate(const orc_basis *B, double *X, int q)
{
    for (int k = (q + 1) * (q + 2) * (q + 3) / 6; k < B->ncoef; ++k) X[k] = 0.0;
}

/* L2L: l_m(c_C) += sum_{k>=m, |k|<=p} C(k,m) (c_C - c_P)^{k-m} l_k(c_P) */
static void orc_l2l_acc(const orc_basis *B, const double *Lp, const double *delta, double *Lc)
{
    double dp[3][ORC_MAXP + 1];
    for (int d = 0; d < 3; ++d) {
        dp[d][0] = 1.0;
        for (int j = 1; j <= B->p; ++j) dp[d][j] = dp[d][j - 1] * delta[d];
    }
    for (int a = 0; a < B->ncoef; ++a) {
        const int *m = B->mi[a];
        double s = 0.0;
        for (int b = 0; b < B->ncoef; ++b) {
            const int *k = B->mi[b];
            if (k[0] < m[0] || k[1] < m[1] || k[2] < m[2]) continue;
            double c = B->binom[k[0]][m[0]] * B->binom[k[1]][m[1]] * B->binom[k[2]][m[2]];
            s += c * dp[0][k[0] - m[0]] * dp[1][k[1] - m[1]] * dp[2][k[2] - m[2]] * Lp[b];
        }
        Lc[a] += s;
    }
}

/* L2P: u(x) = sum_m l_m (x - c)^m */
static double orc_l2p(const orc_basis *B, const double *L, const double *x, const double *c)
{
    double y[3], mono[(ORC_MAXP + 1) * (ORC_MAXP + 2) * (ORC_MAXP + 3) / 6];
    sub3(x, c, y);
    orc_monomials(B, y, mono);
    double s = 0.0;
    for (int k = 0; k < B->ncoef; ++k) s += L[k] * mono[k];
    return s;
}

/* ------------------------------------------------------------------------- */
/* Exported expansion primitives (used by the pin tests).                     */
/* ------------------------------------------------------------------------- */
int orc_ncoef(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }

int orc_multi_indices(int p, int32_t *out)
{
    if (p < 0 || p > ORC_MAXP) return -1;
    orc_basis B;
    orc_basis_init(&B, p);
    for (int k = 0; k < B.ncoef; ++k)
        for (int d = 0; d < 3; ++d) out[3 * k + d] = B.mi[k][d];
    orc_basis_free(&B);
    return 0;
}

int orc_taylor_coeffs(const double *x, int p, double *a)
{
    if (p < 0 || p > ORC_MAXP) return -1;
    orc_basis B;
    orc_basis_init(&B, p);
    orc_taylor(&B, x, p, a);
    orc_basis_free(&B);
    return 0;
}

static int orc_rule_s(int p) { return p / 2; } /* degree 2s+1 >= p */

int orc_p2m_tet(const double *v, const double *M, const double *c, int p, double *Q)
{
    if (p < 0 || p > ORC_MAXP) return -1;
    orc_basis B;
    orc_basis_init(&B, p);
    orc_rule R;
    orc_rule_init(&R, orc_rule_s(p));
    memset(Q, 0, sizeof(double) * (size_t)B.ncoef);
    orc_p2m_tet_acc(&B, &R, v, M, c, Q);
    orc_rule_free(&R);
    orc_basis_free(&B);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Point dipoles, the second source kind of the paper (its "Mag FMM" for      */
/* point-like dipole clouds, Sec. 4).  A dipole of moment m at y is the       */
/* magnetisation m delta(r' - y) in eq. approx1, so                           */
/*   u(x) = m . (x - y) / (4 pi |x - y|^3)   (0 at x = y: no self term)       */
/* and its multipole coefficients (the integral of M . grad'(r' - c)^n) are   */
/*   Q_n = sum_k n_k m_k (y - c)^(n - e_k).                                   */
/* ------------------------------------------------------------------------- */
double orc_dipole_potential(const double *x, const double *y, const double *m)
{
    double d[3];
    sub3(x, y, d);
    const double r2 = dot3(d, d);
    if (r2 == 0.0) return 0.0;
    return ORC_INV4PI * dot3(m, d) / (r2 * sqrt(r2));
}

static void orc_p2m_dipole_acc(const orc_basis *B, const double *y, const double *m, const double *c, double *Q)
{
    double yc[3];
    sub3(y, c, yc);
    double mono[(ORC_MAXP + 1) * (ORC_MAXP + 2) * (ORC_MAXP + 3) / 6];
    orc_monomials(B, yc, mono);
    for (int k = 1; k < B->ncoef; ++k) {
        const int *n = B->mi[k];
        double s = 0.0;
        for (int i = 0; i < 3; ++i) {
            if (n[i] == 0) continue;
            int q[3] = {n[0], n[1], n[2]};
            q[i] -= 1;
            s += n[i] * m[i] * mono[B->idx[q[0]][q[1]][q[2]]];
        }
        Q[k] += s;
    }
}

int orc_p2m_dipole(const double *y, const double *m, const double *c, int p, double *Q)
{
    if (p < 0 || p > ORC_MAXP) return -1;
    orc_basis B;
    orc_basis_init(&B, p);
    memset(Q, 0, sizeof(double) * (size_t)B.ncoef);
    orc_p2m_dipole_acc(&B, y, m, c, Q);
    orc_basis_free(&B);
    return 0;
}

/* O(N^2) dipole sum: pts [n][3], M [F][n][3] moments, targets [nt][3] (NULL: */
/* the points), u [F][nt].                                                     */
int orc_dipole_direct(const double *pts, int64_t n, const double *M, int32_t F, const double *targets, int64_t nt,
                      double *u)
{
    if (!targets) {
        targets = pts;
        nt = n;
    }
    for (int32_t f = 0; f < F; ++f) {
        const double *Mf = M + (size_t)f * n * 3;
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t i = 0; i < nt; ++i) {
            double s = 0.0;
            for (int64_t j = 0; j < n; ++j) s += orc_dipole_potential(targets + 3 * i, pts + 3 * j, Mf + 3 * j);
            u[(size_t)f * nt + i] = s;
        }
    }
    return 0;
}

int orc_m2m(const double *Qc, const double *delta, int p, double *Qp)
{
    if (p < 0 || p > ORC_MAXP) return -1;
    orc_basis B;
    orc_basis_init(&B, p);
    memset(Qp, 0, sizeof(double) * (size_t)B.ncoef);
    orc_m2m_acc(&B, Qc, delta, Qp);
    orc_basis_free(&B);
    return 0;
}

int orc_m2l(const double *Qb, const double *R, int p, double *La)
{
    if (p < 0 || p > ORC_MAXP) return -1;
    orc_basis B;
    orc_basis_init(&B, p);
    memset(La, 0, sizeof(double) * (size_t)B.ncoef);
    orc_m2l_acc(&B, Qb, R, La);
    orc_basis_free(&B);
    return 0;
}

int orc_l2l(const double *Lp, const double *delta, int p, double *Lc)
{
    if (p < 0 || p > ORC_MAXP) return -1;
    orc_basis B;
    orc_basis_init(&B, p);
    memset(Lc, 0, sizeof(double) * (size_t)B.ncoef);
    orc_l2l_acc(&B, Lp, delta, Lc);
    orc_basis_free(&B);
    return 0;
}

int orc_l2p_eval(const double *L, const double *x, const double *c, int p, double *u)
{
    if (p < 0 || p > ORC_MAXP) return -1;
    orc_basis B;
    orc_basis_init(&B, p);
    *u = orc_l2p(&B, L, x, c);
    orc_basis_free(&B);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Octree (Sec. 3.1) over the tets (keyed by centroid) and the targets.       */
/* ------------------------------------------------------------------------- */
typedef struct {
    int level;
    int32_t ix, iy, iz;
    double c[3];
    int parent;
    int child[8];
    int nchild;
    int64_t *tets;
    int64_t ntets;
    int64_t *tgts;
    int64_t ntgts;
    double rsrc, rtgt;
    /* interaction lists with this cell as target */
    int *m2l;
    int nm2l, capm2l;
    int *p2p;
    int np2p, capp2p;
} orc_cell;

typedef struct {
    int64_t n_nodes, n_tets, n_targets;
    double *nodes;   /* [n_nodes][3] */
    int32_t *tetv;   /* [n_tets][4] */
    double *targets; /* [n_targets][3] */
    int p, leaf;
    double theta;
    double origin[3], side;
    uint32_t (*tkey)[3]; /* tet centroid keys at the finest depth */
    uint32_t (*xkey)[3]; /* target keys */
    orc_cell *cells;
    int ncells, capcells;
    int depth;
    int64_t n_m2l, n_p2p, n_p2p_pairs;
    orc_basis B;
    orc_rule R;
    double *Q, *L; /* [ncells][ncoef] for the last evaluated field */
    int points;    /* sources are point dipoles at the nodes (orc_fmm_build_points) */
    int plev[ORC_MAXDEPTH + 1]; /* expansion order of each level (all p by default) */
} orc_fmm;

static uint32_t orc_key1(double xd, double o, double S)
{
    double y = (xd - o) / S;
    double z = floor(y * 2097152.0); /* 2^21 */
    if (z < 0.0) z = 0.0;
    if (z > 2097151.0) z = 2097151.0;
    return (uint32_t)z;
}

static int orc_new_cell(orc_fmm *T)
{
    if (T->ncells == T->capcells) {
        T->capcells = T->capcells ? 2 * T->capcells : 1024;
        T->cells = realloc(T->cells, sizeof(orc_cell) * (size_t)T->capcells);
    }
    orc_cell *C = &T->cells[T->ncells];
    memset(C, 0, sizeof(*C));
    for (int i = 0; i < 8; ++i) C->child[i] = -1;
    C->parent = -1;
    return T->ncells++;
}

static void orc_cell_centre(const orc_fmm *T, int level, int32_t ix, int32_t iy, int32_t iz, double *c)
{
    double s = ldexp(T->side, -level); /* side of a cube at this level */
    c[0] = T->origin[0] + ((double)ix + 0.5) * s;
    c[1] = T->origin[1] + ((double)iy + 0.5) * s;
    c[2] = T->origin[2] + ((double)iz + 0.5) * s;
}

static void orc_split(orc_fmm *T, int ci)
{
    orc_cell *C = &T->cells[ci];
    if (!((C->ntets > T->leaf || C->ntgts > T->leaf) && C->level < ORC_MAXDEPTH)) return;
    int lvl = C->level + 1, sh = ORC_MAXDEPTH - lvl;
    int64_t cntT[8] = {0}, cntX[8] = {0};
    for (int64_t i = 0; i < C->ntets; ++i) {
        const uint32_t *k = T->tkey[C->tets[i]];
        int o = (int)((k[0] >> sh) & 1u) | (int)(((k[1] >> sh) & 1u) << 1) | (int)(((k[2] >> sh) & 1u) << 2);
        cntT[o]++;
    }
    for (int64_t i = 0; i < C->ntgts; ++i) {
        const uint32_t *k = T->xkey[C->tgts[i]];
        int o = (int)((k[0] >> sh) & 1u) | (int)(((k[1] >> sh) & 1u) << 1) | (int)(((k[2] >> sh) & 1u) << 2);
        cntX[o]++;
    }
    for (int o = 0; o < 8; ++o) {
        if (cntT[o] + cntX[o] == 0) continue;
        int ni = orc_new_cell(T);
        C = &T->cells[ci]; /* realloc may move */
        orc_cell *N = &T->cells[ni];
        N->level = lvl;
        N->ix = 2 * C->ix + (o & 1);
        N->iy = 2 * C->iy + ((o >> 1) & 1);
        N->iz = 2 * C->iz + ((o >> 2) & 1);
        orc_cell_centre(T, lvl, N->ix, N->iy, N->iz, N->c);
        N->parent = ci;
        N->tets = malloc(sizeof(int64_t) * (size_t)(cntT[o] ? cntT[o] : 1));
        N->tgts = malloc(sizeof(int64_t) * (size_t)(cntX[o] ? cntX[o] : 1));
        C->child[o] = ni;
        C->nchild++;
    }
    for (int64_t i = 0; i < C->ntets; ++i) {
        const uint32_t *k = T->tkey[C->tets[i]];
        int o = (int)((k[0] >> sh) & 1u) | (int)(((k[1] >> sh) & 1u) << 1) | (int)(((k[2] >> sh) & 1u) << 2);
        orc_cell *N = &T->cells[C->child[o]];
        N->tets[N->ntets++] = C->tets[i];
    }
    for (int64_t i = 0; i < C->ntgts; ++i) {
        const uint32_t *k = T->xkey[C->tgts[i]];
        int o = (int)((k[0] >> sh) & 1u) | (int)(((k[1] >> sh) & 1u) << 1) | (int)(((k[2] >> sh) & 1u) << 2);
        orc_cell *N = &T->cells[C->child[o]];
        N->tgts[N->ntgts++] = C->tgts[i];
    }
    if (lvl > T->depth) T->depth = lvl;
    for (int o = 0; o < 8; ++o)
        if (T->cells[ci].child[o] >= 0) orc_split(T, T->cells[ci].child[o]);
}

static double orc_dist(const double *a, const double *b)
{
    double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return sqrt((dx * dx + dy * dy) + dz * dz);
}

/* Radii of Sec. 3.2: farthest vertex of the cell's tets (source role) and   */
/* farthest target (target role), measured from the cube centre.            */
static void orc_radii(orc_fmm *T)
{
    for (int ci = 0; ci < T->ncells; ++ci) {
        orc_cell *C = &T->cells[ci];
        double rs = 0.0, rt = 0.0;
        for (int64_t i = 0; i < C->ntets; ++i)
            for (int v = 0; v < 4; ++v) {
                double d = orc_dist(T->nodes + 3 * (size_t)T->tetv[4 * C->tets[i] + v], C->c);
                if (d > rs) rs = d;
            }
        for (int64_t i = 0; i < C->ntgts; ++i) {
            double d = orc_dist(T->targets + 3 * C->tgts[i], C->c);
            if (d > rt) rt = d;
        }
        C->rsrc = rs;
        C->rtgt = rt;
    }
}

static void orc_push_list(int **arr, int *n, int *cap, int v)
{
    if (*n == *cap) {
        *cap = *cap ? 2 * *cap : 16;
        *arr = realloc(*arr, sizeof(int) * (size_t)*cap);
    }
    (*arr)[(*n)++] = v;
}

typedef struct {
    int a, b;
} orc_pair;
typedef struct {
    orc_pair *v;
    int64_t n, cap;
} orc_stack;

static void orc_stack_push(orc_stack *S, int a, int b)
{
    if (S->n == S->cap) {
        S->cap = S->cap ? 2 * S->cap : 1024;
        S->v = realloc(S->v, sizeof(orc_pair) * (size_t)S->cap);
    }
    S->v[S->n].a = a;
    S->v[S->n].b = b;
    S->n++;
}

/* MAC (Sec. 3.2): expansion is used iff r_tgt(A) + r_src(B) < theta |c_A - c_B| */
static int orc_mac(const orc_fmm *T, const orc_cell *A, const orc_cell *Bc)
{
    double dx = A->c[0] - Bc->c[0], dy = A->c[1] - Bc->c[1], dz = A->c[2] - Bc->c[2];
    double d2 = (dx * dx + dy * dy) + dz * dz;
    double rr = A->rtgt + Bc->rsrc;
    return rr * rr < (T->theta * T->theta) * d2;
}

/* Interact (Listing 2, with the MAC tested first) */
static void orc_interact(orc_fmm *T, orc_stack *S, int a, int b)
{
    orc_cell *A = &T->cells[a], *Bc = &T->cells[b];
    if (A->ntgts == 0 || Bc->ntets == 0) return;
    if (orc_mac(T, A, Bc)) {
        orc_push_list(&A->m2l, &A->nm2l, &A->capm2l, b);
        T->n_m2l++;
    } else if (A->nchild == 0 && Bc->nchild == 0) {
        orc_push_list(&A->p2p, &A->np2p, &A->capp2p, b);
        T->n_p2p++;
        T->n_p2p_pairs += A->ntgts * Bc->ntets;
    } else {
        orc_stack_push(S, a, b);
    }
}

/* Dual tree traversal (Listing 1) */
static void orc_dtt(orc_fmm *T)
{
    orc_stack S = {0};
    orc_interact(T, &S, 0, 0);
    while (S.n > 0) {
        orc_pair pr = S.v[--S.n];
        const orc_cell *A = &T->cells[pr.a], *Bc = &T->cells[pr.b];
        int splitA = A->level < Bc->level;
        if (splitA && A->nchild == 0) splitA = 0;
        if (!splitA && Bc->nchild == 0) splitA = 1;
        if (splitA) {
            int ch[8];
            for (int o = 0; o < 8; ++o) ch[o] = T->cells[pr.a].child[o];
            for (int o = 0; o < 8; ++o)
                if (ch[o] >= 0) orc_interact(T, &S, ch[o], pr.b);
        } else {
            int ch[8];
            for (int o = 0; o < 8; ++o) ch[o] = T->cells[pr.b].child[o];
            for (int o = 0; o < 8; ++o)
                if (ch[o] >= 0) orc_interact(T, &S, pr.a, ch[o]);
        }
    }
    free(S.v);
}

void orc_fmm_free(void *h);

/* Build the tree and the interaction lists.  targets == NULL means the     */
/* targets are the nodes.  Returns NULL on bad input.                        */
void *orc_fmm_build(const double *nodes, int64_t n_nodes, const int32_t *tets, int64_t n_tets, const double *targets,
                    int64_t n_targets, int32_t p, int32_t leaf, double theta)
{
    if (p < 1 || p > ORC_MAXP || leaf < 1 || !(theta > 0.0 && theta < 1.0) || n_nodes < 1 || n_tets < 1) return NULL;
    for (int64_t t = 0; t < 4 * n_tets; ++t)
        if (tets[t] < 0 || tets[t] >= n_nodes) return NULL;
    orc_fmm *T = calloc(1, sizeof(orc_fmm));
    T->n_nodes = n_nodes;
    T->n_tets = n_tets;
    T->p = p;
    for (int l = 0; l <= ORC_MAXDEPTH; ++l) T->plev[l] = p;
    T->leaf = leaf;
    T->theta = theta;
    T->nodes = malloc(sizeof(double) * 3 * (size_t)n_nodes);
    memcpy(T->nodes, nodes, sizeof(double) * 3 * (size_t)n_nodes);
    T->tetv = malloc(sizeof(int32_t) * 4 * (size_t)n_tets);
    memcpy(T->tetv, tets, sizeof(int32_t) * 4 * (size_t)n_tets);
    if (!targets) {
        targets = nodes;
        n_targets = n_nodes;
    }
    T->n_targets = n_targets;
    T->targets = malloc(sizeof(double) * 3 * (size_t)(n_targets ? n_targets : 1));
    memcpy(T->targets, targets, sizeof(double) * 3 * (size_t)n_targets);

    /* bounding cube: centre of the box of nodes and targets, side = largest
       extent enlarged by 2^-20 */
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) lo[d] = hi[d] = T->nodes[d];
    for (int64_t i = 0; i < n_nodes; ++i)
        for (int d = 0; d < 3; ++d) {
            double q = T->nodes[3 * i + d];
            if (q < lo[d]) lo[d] = q;
            if (q > hi[d]) hi[d] = q;
        }
    for (int64_t i = 0; i < n_targets; ++i)
        for (int d = 0; d < 3; ++d) {
            double q = T->targets[3 * i + d];
            if (q < lo[d]) lo[d] = q;
            if (q > hi[d]) hi[d] = q;
        }
    double ext = 0.0;
    for (int d = 0; d < 3; ++d)
        if (hi[d] - lo[d] > ext) ext = hi[d] - lo[d];
    T->side = ext * (1.0 + ldexp(1.0, -20));
    for (int d = 0; d < 3; ++d) T->origin[d] = (lo[d] + hi[d]) * 0.5 - 0.5 * T->side;

    T->tkey = malloc(sizeof(uint32_t[3]) * (size_t)n_tets);
    for (int64_t t = 0; t < n_tets; ++t) {
        const double *a = T->nodes + 3 * (size_t)tets[4 * t], *b = T->nodes + 3 * (size_t)tets[4 * t + 1];
        const double *c = T->nodes + 3 * (size_t)tets[4 * t + 2], *e = T->nodes + 3 * (size_t)tets[4 * t + 3];
        for (int d = 0; d < 3; ++d) {
            double cen = ((a[d] + b[d]) + (c[d] + e[d])) * 0.25;
            T->tkey[t][d] = orc_key1(cen, T->origin[d], T->side);
        }
    }
    T->xkey = malloc(sizeof(uint32_t[3]) * (size_t)(n_targets ? n_targets : 1));
    for (int64_t i = 0; i < n_targets; ++i)
        for (int d = 0; d < 3; ++d) T->xkey[i][d] = orc_key1(T->targets[3 * i + d], T->origin[d], T->side);

    int root = orc_new_cell(T);
    orc_cell *R = &T->cells[root];
    R->level = 0;
    orc_cell_centre(T, 0, 0, 0, 0, R->c);
    R->ntets = n_tets;
    R->tets = malloc(sizeof(int64_t) * (size_t)n_tets);
    for (int64_t t = 0; t < n_tets; ++t) R->tets[t] = t;
    R->ntgts = n_targets;
    R->tgts = malloc(sizeof(int64_t) * (size_t)(n_targets ? n_targets : 1));
    for (int64_t i = 0; i < n_targets; ++i) R->tgts[i] = i;
    orc_split(T, root);
    orc_radii(T);
    orc_dtt(T);

    orc_basis_init(&T->B, p);
    orc_rule_init(&T->R, orc_rule_s(p));
    return T;
}

/* Tree and lists over point dipoles: source i is the point pts[i], entered  */
/* as a tet whose four corners are that point (centroid and farthest corner   */
/* are the point itself).                                                      */
void *orc_fmm_build_points(const double *pts, int64_t n, const double *targets, int64_t n_targets, int32_t p,
                           int32_t leaf, double theta)
{
    if (n < 1) return NULL;
    int32_t *tv = malloc(sizeof(int32_t) * 4 * (size_t)n);
    for (int64_t i = 0; i < n; ++i)
        for (int c = 0; c < 4; ++c) tv[4 * i + c] = (int32_t)i;
    orc_fmm *T = orc_fmm_build(pts, n, tv, n, targets, n_targets, p, leaf, theta);
    free(tv);
    if (T) T->points = 1;
    return T;
}

void orc_fmm_free(void *h)
{
    orc_fmm *T = h;
    if (!T) return;
    for (int i = 0; i < T->ncells; ++i) {
        free(T->cells[i].tets);
        free(T->cells[i].tgts);
        free(T->cells[i].m2l);
        free(T->cells[i].p2p);
    }
    free(T->cells);
    free(T->nodes);
    free(T->tetv);
    free(T->targets);
    free(T->tkey);
    free(T->xkey);
    free(T->Q);
    free(T->L);
    orc_basis_free(&T->B);
    orc_rule_free(&T->R);
    free(T);
}

/* stats: [ncells, nleaves, depth, n_m2l, n_p2p (cell pairs), n_p2p_pairs (target x tet), ncoef, n_targets] */
void orc_fmm_stats(void *h, int64_t *out)
{
    orc_fmm *T = h;
    int64_t leaves = 0;
    for (int i = 0; i < T->ncells; ++i) leaves += T->cells[i].nchild == 0;
    out[0] = T->ncells;
    out[1] = leaves;
    out[2] = T->depth;
    out[3] = T->n_m2l;
    out[4] = T->n_p2p;
    out[5] = T->n_p2p_pairs;
    out[6] = T->B.ncoef;
    out[7] = T->n_targets;
}

/* Interaction lists as integer cell coordinates:                          */
/* out[8*i..] = levelA, ixA, iyA, izA, levelB, ixB, iyB, izB.                */
/* kind 0 = M2L, 1 = P2P.  out may be NULL to query the count.             */
int64_t orc_fmm_lists(void *h, int32_t kind, int32_t *out)
{
    orc_fmm *T = h;
    int64_t k = 0;
    for (int a = 0; a < T->ncells; ++a) {
        const orc_cell *A = &T->cells[a];
        int n = kind == 0 ? A->nm2l : A->np2p;
        const int *lst = kind == 0 ? A->m2l : A->p2p;
        for (int j = 0; j < n; ++j) {
            if (out) {
                const orc_cell *Bc = &T->cells[lst[j]];
                int32_t *o = out + 8 * k;
                o[0] = A->level;
                o[1] = A->ix;
                o[2] = A->iy;
                o[3] = A->iz;
                o[4] = Bc->level;
                o[5] = Bc->ix;
                o[6] = Bc->iy;
                o[7] = Bc->iz;
            }
            ++k;
        }
    }
    return k;
}

/* Cells: out[6*i..] = level, ix, iy, iz, ntets, ntgts ; radii[2*i..] = rsrc, rtgt */
int64_t orc_fmm_cells(void *h, int32_t *out, double *radii)
{
    orc_fmm *T = h;
    for (int i = 0; i < T->ncells; ++i) {
        const orc_cell *C = &T->cells[i];
        if (out) {
            out[6 * i] = C->level;
            out[6 * i + 1] = C->ix;
            out[6 * i + 2] = C->iy;
            out[6 * i + 3] = C->iz;
            out[6 * i + 4] = (int32_t)C->ntets;
            out[6 * i + 5] = (int32_t)C->ntgts;
        }
        if (radii) {
            radii[2 * i] = C->rsrc;
            radii[2 * i + 1] = C->rtgt;
        }
    }
    return T->ncells;
}

/* Upward pass for one field: P2M at leaves, M2M to the root (post-order). */
static void orc_upward(orc_fmm *T, const double *Mf)
{
    const int nc = T->B.ncoef;
    memset(T->Q, 0, sizeof(double) * (size_t)T->ncells * nc);
#pragma omp parallel for schedule(dynamic, 4)
    for (int ci = 0; ci < T->ncells; ++ci) {
        orc_cell *C = &T->cells[ci];
        if (C->nchild != 0) continue;
        for (int64_t i = 0; i < C->ntets; ++i) {
            if (T->points) {
                const int32_t nd = T->tetv[4 * C->tets[i]];
                orc_p2m_dipole_acc(&T->B, T->nodes + 3 * (size_t)nd, Mf + 3 * (size_t)nd, C->c,
                                   T->Q + (size_t)ci * nc);
                continue;
            }
            double v[12], m[12];
            for (int c = 0; c < 4; ++c) {
                int32_t nd = T->tetv[4 * C->tets[i] + c];
                for (int d = 0; d < 3; ++d) {
                    v[3 * c + d] = T->nodes[3 * (size_t)nd + d];
                    m[3 * c + d] = Mf[3 * (size_t)nd + d];
                }
            }
            orc_p2m_tet_acc(&T->B, &T->R, v, m, C->c, T->Q + (size_t)ci * nc);
        }
    }
    /* children always have larger indices than their parent: sweep backward;
       a cell's multipole is complete when the sweep reaches it and is kept to
       the order of its level (per-level orders) before it is shifted up */
    for (int ci = T->ncells - 1; ci > 0; --ci) {
        orc_cell *C = &T->cells[ci];
        orc_cell *P = &T->cells[C->parent];
        double delta[3];
        orc_truncate(&T->B, T->Q + (size_t)ci * nc, T->plev[C->level]);
        sub3(C->c, P->c, delta);
        orc_m2m_acc(&T->B, T->Q + (size_t)ci * nc, delta, T->Q + (size_t)C->parent * nc);
    }
    if (T->ncells > 0) orc_truncate(&T->B, T->Q, T->plev[0]);
}

static void orc_cell_m2l(orc_fmm *T, int ci)
{
    const int nc = T->B.ncoef;
    orc_cell *A = &T->cells[ci];
    for (int j = 0; j < A->nm2l; ++j) {
        const orc_cell *Bc = &T->cells[A->m2l[j]];
        double R[3];
        sub3(A->c, Bc->c, R);
        orc_m2l_acc_p(&T->B, T->Q + (size_t)A->m2l[j] * nc, R, T->L + (size_t)ci * nc, T->plev[A->level]);
    }
}

/* Near field of one target: P2P with the tets of the leaves in its list. */
static double orc_target_near(const orc_fmm *T, const orc_cell *A, int64_t ti, const double *Mf)
{
    double s = 0.0;
    const double *x = T->targets + 3 * ti;
    for (int j = 0; j < A->np2p; ++j) {
        const orc_cell *Bc = &T->cells[A->p2p[j]];
        for (int64_t i = 0; i < Bc->ntets; ++i) {
            if (T->points) {
                const int32_t nd = T->tetv[4 * Bc->tets[i]];
                s += orc_dipole_potential(x, T->nodes + 3 * (size_t)nd, Mf + 3 * (size_t)nd);
                continue;
            }
            double v[12], m[12];
            for (int c = 0; c < 4; ++c) {
                int32_t nd = T->tetv[4 * Bc->tets[i] + c];
                for (int d = 0; d < 3; ++d) {
                    v[3 * c + d] = T->nodes[3 * (size_t)nd + d];
                    m[3 * c + d] = Mf[3 * (size_t)nd + d];
                }
            }
            s += orc_tet_potential(x, v, m);
        }
    }
    return s;
}

/* Full evaluation: M [F][n_nodes][3] -> u [F][n_targets]. */
int orc_fmm_evaluate(void *h, const double *M, int32_t F, double *u)
{
    orc_fmm *T = h;
    const int nc = T->B.ncoef;
    free(T->Q);
    free(T->L);
    T->Q = malloc(sizeof(double) * (size_t)T->ncells * nc);
    T->L = malloc(sizeof(double) * (size_t)T->ncells * nc);
    for (int32_t f = 0; f < F; ++f) {
        const double *Mf = M + (size_t)f * T->n_nodes * 3;
        double *uf = u + (size_t)f * T->n_targets;
        orc_upward(T, Mf);
        memset(T->L, 0, sizeof(double) * (size_t)T->ncells * nc);
#pragma omp parallel for schedule(dynamic, 4)
        for (int ci = 0; ci < T->ncells; ++ci) orc_cell_m2l(T, ci);
        /* L2L: parents precede children */
        for (int ci = 1; ci < T->ncells; ++ci) {
            orc_cell *C = &T->cells[ci];
            orc_cell *P = &T->cells[C->parent];
            double delta[3];
            sub3(C->c, P->c, delta);
            orc_l2l_acc(&T->B, T->L + (size_t)C->parent * nc, delta, T->L + (size_t)ci * nc);
            orc_truncate(&T->B, T->L + (size_t)ci * nc, T->plev[C->level]);
        }
#pragma omp parallel for schedule(dynamic, 4)
        for (int ci = 0; ci < T->ncells; ++ci) {
            orc_cell *A = &T->cells[ci];
            if (A->nchild != 0) continue;
            for (int64_t i = 0; i < A->ntgts; ++i) {
                int64_t ti = A->tgts[i];
                double far = orc_l2p(&T->B, T->L + (size_t)ci * nc, T->targets + 3 * ti, A->c);
                double near = orc_target_near(T, A, ti, Mf);
                uf[ti] = far + near;
            }
        }
    }
    return 0;
}

/* Evaluation at a subset of targets (indices into the target array).      */
/* The upward pass is done in full; the downward pass only along the paths */
/* from the root to the leaves of the sampled targets.                     */
int orc_fmm_evaluate_sample(void *h, const double *M, int32_t F, const int64_t *sample, int64_t ns, double *u)
{
    orc_fmm *T = h;
    const int nc = T->B.ncoef;
    for (int64_t s = 0; s < ns; ++s)
        if (sample[s] < 0 || sample[s] >= T->n_targets) return -1;
    /* leaf of every target */
    int *leaf_of = malloc(sizeof(int) * (size_t)(T->n_targets ? T->n_targets : 1));
    for (int ci = 0; ci < T->ncells; ++ci) {
        const orc_cell *C = &T->cells[ci];
        if (C->nchild != 0) continue;
        for (int64_t i = 0; i < C->ntgts; ++i) leaf_of[C->tgts[i]] = ci;
    }
    /* mark cells on the root-to-leaf paths */
    char *need = calloc((size_t)(T->ncells > 0 ? T->ncells : 1), 1);
    for (int64_t s = 0; s < ns; ++s)
        for (int c = leaf_of[sample[s]]; c >= 0; c = T->cells[c].parent) need[c] = 1;
    int nneed = 0;
    for (int ci = 0; ci < T->ncells; ++ci) nneed += need[ci];
    int *needlist = malloc(sizeof(int) * (size_t)(nneed ? nneed : 1));
    nneed = 0;
    for (int ci = 0; ci < T->ncells; ++ci)
        if (need[ci]) needlist[nneed++] = ci;

    free(T->Q);
    free(T->L);
    T->Q = malloc(sizeof(double) * (size_t)T->ncells * nc);
    T->L = malloc(sizeof(double) * (size_t)T->ncells * nc);
    for (int32_t f = 0; f < F; ++f) {
        const double *Mf = M + (size_t)f * T->n_nodes * 3;
        orc_upward(T, Mf);
        memset(T->L, 0, sizeof(double) * (size_t)T->ncells * nc);
#pragma omp parallel for schedule(dynamic, 1)
        for (int j = 0; j < nneed; ++j) orc_cell_m2l(T, needlist[j]);
        for (int j = 0; j < nneed; ++j) { /* increasing index: parents first */
            int ci = needlist[j];
            if (ci == 0) continue;
            orc_cell *C = &T->cells[ci];
            double delta[3];
            sub3(C->c, T->cells[C->parent].c, delta);
            orc_l2l_acc(&T->B, T->L + (size_t)C->parent * nc, delta, T->L + (size_t)ci * nc);
            orc_truncate(&T->B, T->L + (size_t)ci * nc, T->plev[C->level]);
        }
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t s = 0; s < ns; ++s) {
            int64_t ti = sample[s];
            int ci = leaf_of[ti];
            const orc_cell *A = &T->cells[ci];
            double far = orc_l2p(&T->B, T->L + (size_t)ci * nc, T->targets + 3 * ti, A->c);
            double near = orc_target_near(T, A, ti, Mf);
            u[(size_t)f * ns + s] = far + near;
        }
    }
    free(leaf_of);
    free(need);
    free(needlist);
    return 0;
}

/* Per-level expansion orders (an accuracy knob beside theta and p): level   */
/* l keeps multipole and local coefficients of degree <= q_l, with          */
/* q_l = order[min(l, n - 1)] clamped to [1, p]; P2M and M2M results are     */
/* truncated at their cell's level, M2L into a cell of level l keeps         */
/* |n| + |m| <= q_l (its sources' multipoles already hold |n| <= q of their  */
/* level), L2L results are truncated at the child's level.  Uniform orders   */
/* (the default) are the method as before.  Returns 0, or -1 on bad input.   */
int orc_fmm_set_level_orders(void *h, const int32_t *order, int32_t n)
{
    orc_fmm *T = h;
    if (!T || !order || n < 1) return -1;
    for (int l = 0; l <= ORC_MAXDEPTH; ++l) {
        int q = order[l < n ? l : n - 1];
        T->plev[l] = q < 1 ? 1 : (q > T->p ? T->p : q);
    }
    return 0;
}

/* After an evaluation: copy the multipole (which=0) or local (which=1)     */
/* coefficients of every cell, in cell order and the graded index order.    */
int orc_fmm_expansions(void *h, int32_t which, double *out)
{
    orc_fmm *T = h;
    const double *src = which == 0 ? T->Q : T->L;
    if (!src) return -1;
    memcpy(out, src, sizeof(double) * (size_t)T->ncells * T->B.ncoef);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Demagnetising field and energy from nodal potentials (the paper's reported */
/* quantity, Sec. 4.1: the stray-field energy of the magnetised box).  With u */
/* interpolated linearly on every tet (P1):                                   */
/*   H_T = -grad u_T = -sum_i u_i grad lambda_i              (per tet)        */
/*   E / mu0 = 1/2 sum_T int_T M . grad u_T = 1/2 sum_T V_T Mbar_T . grad u_T  */
/* (M affine on T, so int_T M = V_T times the mean of its nodal values), and  */
/* the nodal field by mass lumping, the lumped L2 projection of H onto P1:    */
/*   H_j = sum_{T ni j} (V_T / 4) H_T / sum_{T ni j} (V_T / 4).                */
/* nodes [n][3], tets [T][4], M [n][3], u [n]; H_tet [T][3] and H_node [n][3] */
/* may be NULL.  Returns 0, or -1 on a bad index.                             */
/* ------------------------------------------------------------------------- */
int orc_demag(const double *nodes, int64_t n_nodes, const int32_t *tets, int64_t n_tets, const double *M,
              const double *u, double *H_tet, double *H_node, double *energy)
{
    for (int64_t t = 0; t < 4 * n_tets; ++t)
        if (tets[t] < 0 || tets[t] >= n_nodes) return -1;
    double *wsum = NULL;
    if (H_node) {
        wsum = calloc((size_t)(n_nodes > 0 ? n_nodes : 1), sizeof(double));
        for (int64_t j = 0; j < 3 * n_nodes; ++j) H_node[j] = 0.0;
    }
    double E = 0.0;
    for (int64_t t = 0; t < n_tets; ++t) {
        const int32_t *tv = tets + 4 * t;
        const double *V[4] = {nodes + 3 * (size_t)tv[0], nodes + 3 * (size_t)tv[1], nodes + 3 * (size_t)tv[2],
                              nodes + 3 * (size_t)tv[3]};
        double e1[3], e2[3], e3[3], c23[3], c31[3], c12[3];
        sub3(V[1], V[0], e1);
        sub3(V[2], V[0], e2);
        sub3(V[3], V[0], e3);
        cross3(e2, e3, c23);
        cross3(e3, e1, c31);
        cross3(e1, e2, c12);
        const double det = dot3(e1, c23);
        double g[4][3], gu[3] = {0.0, 0.0, 0.0}, mbar[3] = {0.0, 0.0, 0.0};
        for (int d = 0; d < 3; ++d) {
            g[1][d] = c23[d] / det;
            g[2][d] = c31[d] / det;
            g[3][d] = c12[d] / det;
            g[0][d] = -(g[1][d] + g[2][d] + g[3][d]);
        }
        for (int i = 0; i < 4; ++i)
            for (int d = 0; d < 3; ++d) {
                gu[d] += u[tv[i]] * g[i][d];
                mbar[d] += 0.25 * M[3 * (size_t)tv[i] + d];
            }
        const double vol = fabs(det) / 6.0;
        E += 0.5 * vol * dot3(mbar, gu);
        if (H_tet)
            for (int d = 0; d < 3; ++d) H_tet[3 * t + d] = -gu[d];
        if (H_node)
            for (int i = 0; i < 4; ++i) {
                wsum[tv[i]] += 0.25 * vol;
                for (int d = 0; d < 3; ++d) H_node[3 * (size_t)tv[i] + d] -= 0.25 * vol * gu[d];
            }
    }
    if (H_node) {
        for (int64_t j = 0; j < n_nodes; ++j)
            if (wsum[j] > 0.0)
                for (int d = 0; d < 3; ++d) H_node[3 * j + d] /= wsum[j];
        free(wsum);
    }
    *energy = E;
    return 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
