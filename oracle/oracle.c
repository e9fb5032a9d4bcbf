/*
 * Plain FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Method: Ichimura et al., arXiv 2604.02755.
 *   Section 2.1, Eq. 1   Newmark-beta (average acceleration) incremental step
 *   Section 2.1          state updates of q, u, v, a; Rayleigh damping from h;
 *                        second-order tets; absorbing bottom and sides
 *   Section 2.1, Eq. 2   K_e = sum_j w_j B_j^T D_j B_j at the integration points
 *   Section 2.1          multi-spring law, modified Ramberg-Osgood skeleton and
 *                        Masing rule, four doubles and two flags per spring
 *   Section 2.2, Alg. 1  per step: block-Jacobi CRS-PCG, law, CRS update
 *
 * Readings where the paper is silent (each restated where it is used):
 *   4-point degree-2 rule (the text's four evaluation points per tet);
 *   tangent D lagged one step (K^n from D^{n-1});
 *   consistent mass; Lysmer dashpots rho*(Vp nn^T + Vs(I - nn^T)) on base and
 *   side faces; incident-wave input force 2*C_base*v_I;
 *   Rayleigh alpha = a_hat*h, beta = b_hat*h with (a_hat, b_hat) the
 *   least-squares fit of alpha/(4 pi f) + pi beta f to 1 over [f_lo, f_hi];
 *   skeleton e = s(1 + |2s|^beta) with beta = 2 pi h_max / (2 - pi h_max);
 *   Masing branch tau = tau_r + 2 S((gamma - gamma_r)/2), rejoining the
 *   skeleton beyond the largest strain reached; no memory of inner loops;
 *   spring damping h_k = h_max (1 - S(gm)/(G0 gm)), element h = mean;
 *   CG: ||r|| <= tol ||b||, x0 = previous increment.
 */
#include "oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

static double wall_seconds(void)
{
#ifdef _OPENMP
    return omp_get_wtime();
#else
    return 0.0;
#endif
}

void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

static char g_err[512];
const char* or_last_error(void) { return g_err; }
static int fail(int code, const char* msg, long idx)
{
    snprintf(g_err, sizeof g_err, "%s (index %ld)", msg, idx);
    return code;
}

/* 4-point rule: barycentric (a, b, b, b) and permutations, weight V/4. */
static const double QA = 0.5854101966249685;
static const double QB = 0.1381966011250105;
static const int EDGE[6][2] = {{0, 1}, {1, 2}, {2, 0}, {0, 3}, {1, 3}, {2, 3}};

/* ------------------------------------------------------------------ */
/* Geometry and shape functions                                        */
/* ------------------------------------------------------------------ */

/* Barycentric gradients of a straight-sided tet and its volume.
 * x(xi) = x0 + sum_b xi_b (x_b - x0); J_ab = dx_a/dxi_b; grad L_b = row b of J^-1. */
int or_tet_geometry(const double* X, double* gL, double* vol)
{
    double J[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) J[a][b] = X[3 * (b + 1) + a] - X[a];
    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                 J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                 J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    *vol = det / 6.0;
    if (!(det > 0)) return -1;
    double inv[3][3];
    inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    for (int i = 0; i < 3; ++i)
        for (int a = 0; a < 3; ++a) gL[3 * (i + 1) + a] = inv[i][a];
    for (int a = 0; a < 3; ++a) gL[a] = -(gL[3 + a] + gL[6 + a] + gL[9 + a]);
    return 0;
}

/* Gradients of the 10 quadratic shape functions at barycentric point L:
 * corner i: N = L_i(2L_i - 1)  -> (4 L_i - 1) grad L_i
 * edge ab:  N = 4 L_a L_b      -> 4 (L_a grad L_b + L_b grad L_a) */
static void shape_grads(const double L[4], const double* gL, double G[10][3])
{
    for (int i = 0; i < 4; ++i)
        for (int a = 0; a < 3; ++a) G[i][a] = (4.0 * L[i] - 1.0) * gL[3 * i + a];
    for (int e = 0; e < 6; ++e) {
        int p = EDGE[e][0], q = EDGE[e][1];
        for (int a = 0; a < 3; ++a)
            G[4 + e][a] = 4.0 * (L[p] * gL[3 * q + a] + L[q] * gL[3 * p + a]);
    }
}

/* Strain-displacement matrix (6 x 30), Voigt xx, yy, zz, xy, yz, zx with
 * engineering shear. */
static void bmatrix(const double G[10][3], double B[6][30])
{
    memset(B, 0, sizeof(double) * 180);
    for (int n = 0; n < 10; ++n) {
        double gx = G[n][0], gy = G[n][1], gz = G[n][2];
        B[0][3 * n + 0] = gx;
        B[1][3 * n + 1] = gy;
        B[2][3 * n + 2] = gz;
        B[3][3 * n + 0] = gy; B[3][3 * n + 1] = gx;
        B[4][3 * n + 1] = gz; B[4][3 * n + 2] = gy;
        B[5][3 * n + 2] = gx; B[5][3 * n + 0] = gz;
    }
}

static void ip_bary(int j, double L[4])
{
    for (int i = 0; i < 4; ++i) L[i] = (i == j) ? QA : QB;
}

static double fact(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= (double)i;
    return f;
}

/* Quadratic shape functions as sums of barycentric monomials. */
typedef struct { int nterm; double c[2]; int ex[2][4]; } poly;
static void shape_poly(int n, poly* P)
{
    memset(P, 0, sizeof *P);
    if (n < 4) { /* 2 L_i^2 - L_i */
        P->nterm = 2;
        P->c[0] = 2.0; P->ex[0][n] = 2;
        P->c[1] = -1.0; P->ex[1][n] = 1;
    } else { /* 4 L_a L_b */
        P->nterm = 1;
        P->c[0] = 4.0;
        P->ex[0][EDGE[n - 4][0]] += 1;
        P->ex[0][EDGE[n - 4][1]] += 1;
    }
}

/* Reference consistent mass: Mref[a][b] = (1/V) int N_a N_b dV, from
 * int L1^p L2^q L3^r L4^s dV = 6V p! q! r! s! / (p+q+r+s+3)!. */
static void mass_ref(double Mref[10][10])
{
    for (int a = 0; a < 10; ++a)
        for (int b = 0; b < 10; ++b) {
            poly A, Bp;
            shape_poly(a, &A);
            shape_poly(b, &Bp);
            double s = 0.0;
            for (int i = 0; i < A.nterm; ++i)
                for (int j = 0; j < Bp.nterm; ++j) {
                    int e[4], tot = 0;
                    double num = 1.0;
                    for (int k = 0; k < 4; ++k) {
                        e[k] = A.ex[i][k] + Bp.ex[j][k];
                        tot += e[k];
                        num *= fact(e[k]);
                    }
                    s += A.c[i] * Bp.c[j] * 6.0 * num / fact(tot + 3);
                }
            Mref[a][b] = s;
        }
}

/* Element stiffness (Eq. 2) with the 4-point rule and consistent mass.
 * D4x36: full 6x6 D at each of the 4 points.  Outputs 30x30 row-major with
 * local DOF 3*node + component. */
void or_element_matrices(const double* X, const double* D4x36, double rho, double* Ke,
                         double* Me)
{
    double gL[12], V;
    or_tet_geometry(X, gL, &V);
    if (Ke) {
        memset(Ke, 0, sizeof(double) * 900);
        for (int j = 0; j < 4; ++j) {
            double L[4], G[10][3], B[6][30], DB[6][30];
            ip_bary(j, L);
            shape_grads(L, gL, G);
            bmatrix(G, B);
            const double* D = D4x36 + 36 * j;
            for (int r = 0; r < 6; ++r)
                for (int c = 0; c < 30; ++c) {
                    double s = 0.0;
                    for (int k = 0; k < 6; ++k) s += D[6 * r + k] * B[k][c];
                    DB[r][c] = s;
                }
            for (int a = 0; a < 30; ++a)
                for (int b = 0; b < 30; ++b) {
                    double s = 0.0;
                    for (int k = 0; k < 6; ++k) s += B[k][a] * DB[k][b];
                    Ke[30 * a + b] += 0.25 * V * s;
                }
        }
    }
    if (Me) {
        double Mref[10][10];
        mass_ref(Mref);
        memset(Me, 0, sizeof(double) * 900);
        for (int a = 0; a < 10; ++a)
            for (int b = 0; b < 10; ++b)
                for (int c = 0; c < 3; ++c) Me[30 * (3 * a + c) + 3 * b + c] = rho * V * Mref[a][b];
    }
}

/* 6-node triangle: M36[a][b] = int N_a N_b dA (corners lambda(2 lambda - 1),
 * edges 4 lambda_a lambda_b), from int l1^p l2^q l3^r dA = 2A p!q!r!/(p+q+r+2)!. */
void or_face_matrix(const double* X, double* M, double* nrm, double* area)
{
    double e1[3], e2[3], c[3];
    for (int a = 0; a < 3; ++a) {
        e1[a] = X[3 + a] - X[a];
        e2[a] = X[6 + a] - X[a];
    }
    c[0] = e1[1] * e2[2] - e1[2] * e2[1];
    c[1] = e1[2] * e2[0] - e1[0] * e2[2];
    c[2] = e1[0] * e2[1] - e1[1] * e2[0];
    double n2 = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    double A = 0.5 * n2;
    for (int a = 0; a < 3; ++a) nrm[a] = c[a] / n2;
    *area = A;
    static const int FE[3][2] = {{0, 1}, {1, 2}, {2, 0}};
    for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b) {
            /* expand N_a N_b into monomials of (l1, l2, l3) */
            double ca[2], cb[2];
            int ea[2][3] = {{0}}, eb[2][3] = {{0}}, na, nb;
            if (a < 3) { na = 2; ca[0] = 2; ea[0][a] = 2; ca[1] = -1; ea[1][a] = 1; }
            else { na = 1; ca[0] = 4; ea[0][FE[a - 3][0]] = 1; ea[0][FE[a - 3][1]] = 1; }
            if (b < 3) { nb = 2; cb[0] = 2; eb[0][b] = 2; cb[1] = -1; eb[1][b] = 1; }
            else { nb = 1; cb[0] = 4; eb[0][FE[b - 3][0]] = 1; eb[0][FE[b - 3][1]] = 1; }
            double s = 0.0;
            for (int i = 0; i < na; ++i)
                for (int j = 0; j < nb; ++j) {
                    int tot = 0;
                    double num = 1.0;
                    for (int k = 0; k < 3; ++k) {
                        int e = ea[i][k] + eb[j][k];
                        tot += e;
                        num *= fact(e);
                    }
                    s += ca[i] * cb[j] * 2.0 * A * num / fact(tot + 2);
                }
            M[6 * a + b] = s;
        }
}

/* Least-squares Rayleigh fit: minimise int_{f_lo}^{f_hi} (a/(4 pi f) + pi b f - 1)^2 df. */
void or_rayleigh(double fl, double fh, double* ah, double* bh)
{
    const double pi = M_PI;
    double m11 = (1.0 / fl - 1.0 / fh) / (16.0 * pi * pi);
    double m12 = (fh - fl) / 4.0;
    double m22 = pi * pi * (fh * fh * fh - fl * fl * fl) / 3.0;
    double r1 = log(fh / fl) / (4.0 * pi);
    double r2 = pi * (fh * fh - fl * fl) / 2.0;
    double det = m11 * m22 - m12 * m12;
    *ah = (r1 * m22 - m12 * r2) / det;
    *bh = (m11 * r2 - m12 * r1) / det;
}

/* ------------------------------------------------------------------ */
/* Spring law                                                          */
/* ------------------------------------------------------------------ */

double or_ro_beta(double h_max) { return 2.0 * M_PI * h_max / (2.0 - M_PI * h_max); }

/* s with s (1 + |2s|^beta) = e, by Newton from an upper bound. */
double or_ro_inverse(double e, double beta)
{
    double a = fabs(e);
    if (a == 0.0) return 0.0;
    double s = fmin(a, pow(a / pow(2.0, beta), 1.0 / (1.0 + beta)));
    for (int it = 0; it < 60; ++it) {
        double p = pow(2.0 * s, beta);
        double f = s * (1.0 + p) - a;
        if (f <= 0.0) break;
        double ds = f / (1.0 + (1.0 + beta) * p);
        s -= ds;
        if (ds <= 0x1p-52 * s) break;
    }
    return e < 0 ? -s : s;
}

typedef struct { double G0, gref, hmax, beta; } spring_par;

/* skeleton stress S(gamma) = G0 gref s(gamma/gref) */
static double skeleton(double g, const spring_par* p)
{
    return p->G0 * p->gref * or_ro_inverse(g / p->gref, p->beta);
}

static double stress_on_curve(double g, const double* st, const spring_par* p)
{
    if (st[5] != 0.0) return skeleton(g, p);
    return st[2] + 2.0 * skeleton(0.5 * (g - st[1]), p);
}

/* state: gp (current strain), gr (reversal strain), tr (reversal stress),
 * gm (largest |strain| on the skeleton), dir (last loading sign), skel (on skeleton).
 * With a memory of depth K > 1 (the last K reversal points: the current
 * branch's origin and K - 1 older ones) the record goes on with the count of
 * older points and up to K - 1 of them as (gr, tr) pairs, the most recent
 * last: st[6] = count, st[7 + 2i], st[8 + 2i].  Depth 1 is the three-rule law
 * (skeleton, Masing branch from the last reversal, rejoin beyond the largest
 * strain reached).  Depth K adds the rule that closes inner loops: a branch
 * that reaches the reversal point where the previous branch began continues
 * on the branch before that one (the two reversal points are forgotten), so
 * loops nested up to K - 2 deep close (depth 2 behaves as depth 1); when
 * K - 1 older points are held the oldest is dropped, and a loop that lost
 * its outer point ends only by the rejoin.
 * cnt (optional) counts the events of the step for the tests: [0] reversals
 * taken on the skeleton, [1] reversals taken on a Masing branch, [2] rejoins
 * of the skeleton, [3] inner loops closed. */
static void spring_update(double* st, double dg, const spring_par* p, int depth, double* Gt, double* hk, long* cnt)
{
    if (dg != 0.0) {
        double d = dg > 0.0 ? 1.0 : -1.0;
        if (st[4] != 0.0 && d != st[4]) { /* reversal: branch starts at the current point */
            if (cnt) cnt[st[5] != 0.0 ? 0 : 1]++;
            const double trev = stress_on_curve(st[0], st, p);
            if (depth > 1 && st[5] == 0.0) { /* keep the origin of the branch being left */
                int k = (int)st[6];
                if (k == depth - 1) { /* full: drop the oldest point */
                    for (int i = 0; i + 1 < k; ++i) {
                        st[7 + 2 * i] = st[9 + 2 * i];
                        st[8 + 2 * i] = st[10 + 2 * i];
                    }
                    --k;
                }
                st[7 + 2 * k] = st[1];
                st[8 + 2 * k] = st[2];
                st[6] = k + 1;
            }
            st[2] = trev;
            st[1] = st[0];
            st[5] = 0.0;
        }
        st[4] = d;
        double g = st[0] + dg;
        if (st[5] == 0.0 && d * g >= st[3]) { /* back on the skeleton beyond every loop */
            st[5] = 1.0;
            if (depth > 1) st[6] = 0.0;
            if (cnt) cnt[2]++;
        }
        /* a closed inner loop: on to the branch before the previous one */
        while (depth > 1 && st[5] == 0.0 && st[6] >= 2.0 && d * g >= d * st[7 + 2 * ((int)st[6] - 1)]) {
            const int k = (int)st[6];
            st[1] = st[7 + 2 * (k - 2)];
            st[2] = st[8 + 2 * (k - 2)];
            st[6] = k - 2;
            if (cnt) cnt[3]++;
        }
        if (st[5] != 0.0) st[3] = fmax(st[3], fabs(g));
        st[0] = g;
    }
    double xi = st[5] != 0.0 ? st[0] : 0.5 * (st[0] - st[1]);
    double s = or_ro_inverse(xi / p->gref, p->beta);
    *Gt = p->G0 / (1.0 + (1.0 + p->beta) * pow(fabs(2.0 * s), p->beta));
    if (st[3] > 0.0) {
        double em = st[3] / p->gref;
        *hk = p->hmax * (1.0 - or_ro_inverse(em, p->beta) / em);
    } else {
        *hk = 0.0;
    }
}

double or_spring_step(double* st, double dg, double G0, double gref, double h_max, double* Gt,
                      double* hk)
{
    spring_par p = {G0, gref, h_max, or_ro_beta(h_max)};
    spring_update(st, dg, &p, 1, Gt, hk, NULL);
    return stress_on_curve(st[0], st, &p);
}

double or_spring_step_mem(double* st, int depth, double dg, double G0, double gref, double h_max, double* Gt,
                          double* hk, long* events)
{
    spring_par p = {G0, gref, h_max, or_ro_beta(h_max)};
    spring_update(st, dg, &p, depth, Gt, hk, events);
    return stress_on_curve(st[0], st, &p);
}

int or_spring_words(int depth) { return depth > 1 ? 5 + 2 * depth : 6; }

/* Multi-spring point: D = Kb m m^T + sum_k c_k G_t,k n_k n_k^T, h = mean h_k.
 * cnt (optional): law events, as for spring_update. */
static void ip_law(const double* deps, double* state, int ns, int depth, const double* dirs, const double* w,
                   double G0, double Kb, double gref, double hmax, double* D, double* hmean, long* cnt)
{
    const int sw = or_spring_words(depth);
    spring_par p = {G0, gref, hmax, or_ro_beta(hmax)};
    for (int i = 0; i < 36; ++i) D[i] = 0.0;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) D[6 * r + c] = Kb;
    double hs = 0.0;
    for (int k = 0; k < ns; ++k) {
        const double* n = dirs + 6 * k;
        double Gt = G0, hk = 0.0;
        if (deps) { /* deps == NULL: the initial (virgin) tangent G0 */
            double dg = 0.0;
            for (int i = 0; i < 6; ++i) dg += n[i] * deps[i];
            spring_update(state + (long)sw * k, dg, &p, depth, &Gt, &hk, cnt);
        }
        for (int r = 0; r < 6; ++r)
            for (int c = 0; c < 6; ++c) D[6 * r + c] += w[k] * Gt * n[r] * n[c];
        hs += hk;
    }
    *hmean = hs / ns;
}

void or_ip_law(const double* deps, double* state, int ns, const double* dirs, const double* w,
               double G0, double Kb, double gref, double hmax, double* D, double* hmean)
{
    ip_law(deps, state, ns, 1, dirs, w, G0, Kb, gref, hmax, D, hmean, NULL);
}

/* ------------------------------------------------------------------ */
/* Block-CRS system                                                    */
/* ------------------------------------------------------------------ */

typedef struct {
    int nn;        /* nodes */
    int* rowptr;   /* [nn+1] */
    int* col;      /* [nnzb] */
    int nnzb;
} pattern;

static int cmp_int(const void* a, const void* b)
{
    int x = *(const int*)a, y = *(const int*)b;
    return (x > y) - (x < y);
}

static int build_pattern(int nn, int ne, const int* conn /* [ne*10], aliased */, pattern* P)
{
    /* count incidences */
    int* cnt = calloc((size_t)nn + 1, sizeof(int));
    if (!cnt) return -1;
    for (long e = 0; e < ne; ++e)
        for (int a = 0; a < 10; ++a) cnt[conn[10 * e + a]] += 10;
    long* start = malloc(sizeof(long) * ((size_t)nn + 1));
    start[0] = 0;
    for (int i = 0; i < nn; ++i) start[i + 1] = start[i] + cnt[i];
    int* buf = malloc(sizeof(int) * (size_t)start[nn]);
    long* fill = calloc((size_t)nn, sizeof(long));
    for (long e = 0; e < ne; ++e)
        for (int a = 0; a < 10; ++a) {
            int r = conn[10 * e + a];
            for (int b = 0; b < 10; ++b) buf[start[r] + fill[r]++] = conn[10 * e + b];
        }
    P->nn = nn;
    P->rowptr = malloc(sizeof(int) * ((size_t)nn + 1));
    long tot = 0;
    for (int i = 0; i < nn; ++i) {
        int* row = buf + start[i];
        int m = (int)(start[i + 1] - start[i]);
        qsort(row, m, sizeof(int), cmp_int);
        int u = 0;
        for (int k = 0; k < m; ++k)
            if (k == 0 || row[k] != row[k - 1]) row[u++] = row[k];
        cnt[i] = u;
        tot += u;
    }
    P->nnzb = (int)tot;
    P->col = malloc(sizeof(int) * (size_t)tot);
    P->rowptr[0] = 0;
    for (int i = 0; i < nn; ++i) {
        memcpy(P->col + P->rowptr[i], buf + start[i], sizeof(int) * cnt[i]);
        P->rowptr[i + 1] = P->rowptr[i] + cnt[i];
    }
    free(cnt);
    free(start);
    free(buf);
    free(fill);
    return 0;
}

static int find_block(const pattern* P, int r, int c)
{
    int lo = P->rowptr[r], hi = P->rowptr[r + 1] - 1;
    while (lo <= hi) {
        int mid = (lo + hi) / 2;
        if (P->col[mid] == c) return mid;
        if (P->col[mid] < c) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* add a 30x30 (or 18x18 for faces) element matrix scaled by s */
static void scatter(const pattern* P, double* blocks, const int* nodes, int nloc,
                    const double* Me, double s)
{
    int n3 = 3 * nloc;
    for (int a = 0; a < nloc; ++a)
        for (int b = 0; b < nloc; ++b) {
            int k = find_block(P, nodes[a], nodes[b]);
            double* blk = blocks + 9 * (long)k;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) blk[3 * i + j] += s * Me[n3 * (3 * a + i) + 3 * b + j];
        }
}

static void spmv(const pattern* P, const double* blocks, const double* x, double* y)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < P->nn; ++i) {
        double s0 = 0, s1 = 0, s2 = 0;
        for (int k = P->rowptr[i]; k < P->rowptr[i + 1]; ++k) {
            const double* b = blocks + 9 * (long)k;
            const double* xv = x + 3 * (long)P->col[k];
            s0 += b[0] * xv[0] + b[1] * xv[1] + b[2] * xv[2];
            s1 += b[3] * xv[0] + b[4] * xv[1] + b[5] * xv[2];
            s2 += b[6] * xv[0] + b[7] * xv[1] + b[8] * xv[2];
        }
        y[3 * i] = s0;
        y[3 * i + 1] = s1;
        y[3 * i + 2] = s2;
    }
}

static double dot(long n, const double* a, const double* b)
{
    double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (long i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

static int inv3(const double* a, double* o)
{
    double det = a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
                 a[2] * (a[3] * a[7] - a[4] * a[6]);
    if (det == 0.0) {
        memset(o, 0, sizeof(double) * 9);
        return -1;
    }
    o[0] = (a[4] * a[8] - a[5] * a[7]) / det;
    o[1] = (a[2] * a[7] - a[1] * a[8]) / det;
    o[2] = (a[1] * a[5] - a[2] * a[4]) / det;
    o[3] = (a[5] * a[6] - a[3] * a[8]) / det;
    o[4] = (a[0] * a[8] - a[2] * a[6]) / det;
    o[5] = (a[2] * a[3] - a[0] * a[5]) / det;
    o[6] = (a[3] * a[7] - a[4] * a[6]) / det;
    o[7] = (a[1] * a[6] - a[0] * a[7]) / det;
    o[8] = (a[0] * a[4] - a[1] * a[3]) / det;
    return 0;
}

/* 3x3 block-Jacobi preconditioned CG (Section 2.2, Algorithm 1's CRS-PCG).
 * Solves A x = b from the given x; stops when ||r|| <= tol ||b||. */
static int pcg(const pattern* P, const double* A, const double* b, double* x, double tol, int maxit,
               int* iters)
{
    long n = 3L * P->nn;
    double* Pinv = malloc(sizeof(double) * 9 * (size_t)P->nn);
    double* r = malloc(sizeof(double) * n);
    double* z = malloc(sizeof(double) * n);
    double* p = malloc(sizeof(double) * n);
    double* q = malloc(sizeof(double) * n);
    for (int i = 0; i < P->nn; ++i) {
        int k = find_block(P, i, i);
        if (k < 0 || inv3(A + 9 * (long)k, Pinv + 9 * (long)i) != 0)
            memset(Pinv + 9 * (long)i, 0, sizeof(double) * 9); /* node without DOFs */
    }
    double bn = sqrt(dot(n, b, b));
    int it = 0, rc = 0;
    if (bn == 0.0) {
        memset(x, 0, sizeof(double) * n);
        goto done;
    }
    spmv(P, A, x, q);
    for (long i = 0; i < n; ++i) r[i] = b[i] - q[i];
    double rn = sqrt(dot(n, r, r));
    if (rn <= tol * bn) goto done;
    for (int i = 0; i < P->nn; ++i) {
        const double* m = Pinv + 9 * (long)i;
        const double* rv = r + 3L * i;
        for (int c = 0; c < 3; ++c) z[3L * i + c] = m[3 * c] * rv[0] + m[3 * c + 1] * rv[1] + m[3 * c + 2] * rv[2];
    }
    memcpy(p, z, sizeof(double) * n);
    double rz = dot(n, r, z);
    for (it = 1; it <= maxit; ++it) {
        spmv(P, A, p, q);
        double alpha = rz / dot(n, p, q);
        for (long i = 0; i < n; ++i) {
            x[i] += alpha * p[i];
            r[i] -= alpha * q[i];
        }
        rn = sqrt(dot(n, r, r));
        if (rn <= tol * bn) break;
        for (int i = 0; i < P->nn; ++i) {
            const double* m = Pinv + 9 * (long)i;
            const double* rv = r + 3L * i;
            for (int c = 0; c < 3; ++c)
                z[3L * i + c] = m[3 * c] * rv[0] + m[3 * c + 1] * rv[1] + m[3 * c + 2] * rv[2];
        }
        double rz1 = dot(n, r, z);
        double beta = rz1 / rz;
        rz = rz1;
        for (long i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    }
    if (it > maxit) {
        it = maxit;
        rc = -1;
    }
done:
    *iters = it;
    free(Pinv);
    free(r);
    free(z);
    free(p);
    free(q);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Driver: Algorithm 1 in FP64                                         */
/* ------------------------------------------------------------------ */

typedef struct { int key[3]; int tet; } face_key;
static int cmp_face(const void* a, const void* b)
{
    const face_key* x = a;
    const face_key* y = b;
    for (int i = 0; i < 3; ++i)
        if (x->key[i] != y->key[i]) return x->key[i] < y->key[i] ? -1 : 1;
    return 0;
}
static void sort3(int* k)
{
    if (k[0] > k[1]) { int t = k[0]; k[0] = k[1]; k[1] = t; }
    if (k[1] > k[2]) { int t = k[1]; k[1] = k[2]; k[2] = t; }
    if (k[0] > k[1]) { int t = k[0]; k[0] = k[1]; k[1] = t; }
}

int or_run(const or_mesh* m, const or_problem* pr, or_result* res)
{
    const int nn = m->n_nodes, ne = m->n_tets, ns = pr->n_springs;
    const long ndof = 3L * nn;
    const double dt = pr->dt;
    const double t_start = wall_seconds();
    res->steps_done = 0;
    res->setup_seconds = 0.0;
    res->law_events[0] = res->law_events[1] = res->law_events[2] = res->law_events[3] = 0;
    if (res->vmax)
        for (int r = 0; r < m->n_recv; ++r) res->vmax[r] = 0.0;

    /* --- validate the mesh --- */
    for (long i = 0; i < 10L * ne; ++i)
        if (m->tet10[i] < 0 || m->tet10[i] >= nn) return fail(OR_EINVAL, "node index out of range", i / 10);
    for (long e = 0; e < ne; ++e)
        if (m->layer[e] < 0 || m->layer[e] >= pr->n_layers) return fail(OR_EINVAL, "layer out of range", e);

    int* conn = malloc(sizeof(int) * 10 * (size_t)ne);
    for (long i = 0; i < 10L * ne; ++i) conn[i] = m->alias ? m->alias[m->tet10[i]] : m->tet10[i];

    /* --- per-element geometry --- */
    double* gLall = malloc(sizeof(double) * 12 * (size_t)ne);
    double* vol = malloc(sizeof(double) * (size_t)ne);
    double* Xall = malloc(sizeof(double) * 12 * (size_t)ne);
    for (long e = 0; e < ne; ++e) {
        double* X = Xall + 12 * e;
        for (int a = 0; a < 4; ++a)
            for (int c = 0; c < 3; ++c) X[3 * a + c] = m->xyz[3L * m->tet10[10 * e + a] + c];
        if (or_tet_geometry(X, gLall + 12 * e, vol + e) != 0) {
            free(conn); free(gLall); free(vol); free(Xall);
            return fail(OR_EINVAL, "non-positive Jacobian", e);
        }
        for (int k = 0; k < 6; ++k) {
            const double* pa = m->xyz + 3L * m->tet10[10 * e + EDGE[k][0]];
            const double* pb = m->xyz + 3L * m->tet10[10 * e + EDGE[k][1]];
            const double* pm = m->xyz + 3L * m->tet10[10 * e + 4 + k];
            double el = 0.0, dv = 0.0;
            for (int c = 0; c < 3; ++c) {
                el += (pb[c] - pa[c]) * (pb[c] - pa[c]);
                double d = pm[c] - 0.5 * (pa[c] + pb[c]);
                dv += d * d;
            }
            if (dv > 1e-18 * el) {
                free(conn); free(gLall); free(vol); free(Xall);
                return fail(OR_EINVAL, "curved edge (mid-node off the midpoint)", e);
            }
        }
    }

    /* --- materials per layer --- */
    int nl = pr->n_layers;
    double *G0 = malloc(sizeof(double) * nl), *Kb = malloc(sizeof(double) * nl),
           *vp = malloc(sizeof(double) * nl);
    for (int l = 0; l < nl; ++l) {
        double rho = pr->rho[l], vs = pr->vs[l], nu = pr->nu[l];
        G0[l] = rho * vs * vs;
        double lam = 2.0 * G0[l] * nu / (1.0 - 2.0 * nu);
        Kb[l] = lam + 2.0 * G0[l] / 3.0;
        vp[l] = sqrt((lam + 2.0 * G0[l]) / rho);
    }

    pattern P;
    build_pattern(nn, ne, conn, &P);
    size_t nb = (size_t)P.nnzb * 9;
    double* Mg = calloc(nb, sizeof(double));
    double* Kg = calloc(nb, sizeof(double));
    double* Cg = calloc(nb, sizeof(double));
    double* Cabs = calloc(nb, sizeof(double));
    double* Ag = calloc(nb, sizeof(double));
    if (!Mg || !Kg || !Cg || !Cabs || !Ag) return fail(OR_ENOMEM, "out of memory", 0);

    /* --- constant mass --- */
    {
        double Me[900];
        for (long e = 0; e < ne; ++e) {
            or_element_matrices(Xall + 12 * e, NULL, pr->rho[m->layer[e]], NULL, Me);
            scatter(&P, Mg, conn + 10 * e, 10, Me, 1.0);
        }
    }

    /* --- absorbing faces: dashpot rho (Vp n n^T + Vs (I - n n^T)) --- */
    double* Wbase = calloc((size_t)ndof * 3, sizeof(double)); /* per node: sum_j C_base,ij (3x3) */
    {
        face_key* fk = malloc(sizeof(face_key) * 4 * (size_t)ne);
        static const int TF[4][3] = {{0, 1, 2}, {1, 2, 3}, {0, 2, 3}, {0, 1, 3}};
        for (long e = 0; e < ne; ++e)
            for (int f = 0; f < 4; ++f) {
                face_key* k = fk + 4 * e + f;
                for (int i = 0; i < 3; ++i) k->key[i] = m->tet10[10 * e + TF[f][i]];
                sort3(k->key);
                k->tet = (int)e;
            }
        qsort(fk, 4 * (size_t)ne, sizeof(face_key), cmp_face);
        for (long f = 0; f < m->n_bfaces; ++f) {
            const int* fn = m->bface6 + 6 * f;
            face_key q;
            for (int i = 0; i < 3; ++i) q.key[i] = fn[i];
            sort3(q.key);
            face_key* hit = bsearch(&q, fk, 4 * (size_t)ne, sizeof(face_key), cmp_face);
            if (!hit) {
                free(fk);
                return fail(OR_EINVAL, "boundary face not on any tet", f);
            }
            int l = m->layer[hit->tet];
            double X[9], M36[36], nv[3], A;
            for (int i = 0; i < 3; ++i)
                for (int c = 0; c < 3; ++c) X[3 * i + c] = m->xyz[3L * fn[i] + c];
            or_face_matrix(X, M36, nv, &A);
            double Z[9];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j)
                    Z[3 * i + j] = pr->rho[l] * (vp[l] * nv[i] * nv[j] + pr->vs[l] * ((i == j) - nv[i] * nv[j]));
            double C18[324];
            for (int a = 0; a < 6; ++a)
                for (int b = 0; b < 6; ++b)
                    for (int i = 0; i < 3; ++i)
                        for (int j = 0; j < 3; ++j) C18[18 * (3 * a + i) + 3 * b + j] = M36[6 * a + b] * Z[3 * i + j];
            int fa[6];
            for (int i = 0; i < 6; ++i) fa[i] = m->alias ? m->alias[fn[i]] : fn[i];
            scatter(&P, Cabs, fa, 6, C18, 1.0);
            if (m->bface_kind[f] == 0)
                for (int a = 0; a < 6; ++a)
                    for (int b = 0; b < 6; ++b)
                        for (int k = 0; k < 9; ++k) Wbase[9L * fa[a] + k] += M36[6 * a + b] * Z[k];
        }
        free(fk);
    }

    /* --- state --- */
    double* D = malloc(sizeof(double) * 36 * 4 * (size_t)ne);
    const int depth = pr->masing_depth > 1 ? pr->masing_depth : 1;
    const int sw = or_spring_words(depth);
    double* th = calloc((size_t)ne * 4 * ns * sw, sizeof(double));
    double* he = calloc((size_t)ne, sizeof(double));
    for (long i = 0; i < (long)ne * 4 * ns; ++i) th[sw * i + 5] = 1.0; /* start on the skeleton */
    for (long e = 0; e < ne; ++e) {
        int l = m->layer[e];
        for (int j = 0; j < 4; ++j) {
            double hm;
            or_ip_law(NULL, NULL, ns, pr->dirs, pr->weights, G0[l], Kb[l], pr->gamma_ref[l], pr->h_max[l],
                      D + 36 * (4 * e + j), &hm);
        }
    }
    double ahat = 0.0, bhat = 0.0;
    if (pr->damping_mode != 2) or_rayleigh(pr->f_lo, pr->f_hi, &ahat, &bhat);

    if (pr->apply_which >= 0) { /* operator application with the given D and h */
        for (long i = 0; i < 4L * ne; ++i) {
            int k = 0;
            for (int r = 0; r < 6; ++r)
                for (int c = r; c < 6; ++c) {
                    D[36 * i + 6 * r + c] = pr->apply_D[21 * i + k];
                    D[36 * i + 6 * c + r] = pr->apply_D[21 * i + k];
                    ++k;
                }
        }
        double Ke[900], Me[900];
        memcpy(Cg, Cabs, nb * sizeof(double));
        for (long e = 0; e < ne; ++e) {
            double h = pr->damping_mode == 0 ? (pr->apply_h ? pr->apply_h[e] : 0.0)
                                             : (pr->damping_mode == 1 ? pr->h0 : 0.0);
            or_element_matrices(Xall + 12 * e, D + 144 * e, pr->rho[m->layer[e]], Ke, Me);
            scatter(&P, Kg, conn + 10 * e, 10, Ke, 1.0);
            if (h != 0.0) {
                scatter(&P, Cg, conn + 10 * e, 10, Me, ahat * h);
                scatter(&P, Cg, conn + 10 * e, 10, Ke, bhat * h);
            }
        }
        for (size_t k = 0; k < nb; ++k)
            Ag[k] = pr->apply_which == 0 ? 4.0 / (dt * dt) * Mg[k] + 2.0 / dt * Cg[k] + Kg[k]
                  : (pr->apply_which == 1 ? Kg[k] : Mg[k]);
        spmv(&P, Ag, pr->apply_x, pr->apply_y);
        free(D); free(th); free(he); free(Wbase);
        free(Mg); free(Kg); free(Cg); free(Cabs); free(Ag);
        free(P.rowptr); free(P.col);
        free(G0); free(Kb); free(vp);
        free(conn); free(gLall); free(vol); free(Xall);
        return OR_OK;
    }

    double *u = calloc(ndof, sizeof(double)), *v = calloc(ndof, sizeof(double)),
           *acc = calloc(ndof, sizeof(double)), *q = calloc(ndof, sizeof(double)),
           *du = calloc(ndof, sizeof(double)), *b = calloc(ndof, sizeof(double)),
           *t1 = calloc(ndof, sizeof(double)), *t2 = calloc(ndof, sizeof(double));
    double vI[3] = {0, 0, 0}, aprev[3] = {0, 0, 0};
    int rc = OR_OK;
    if (pr->v0) memcpy(v, pr->v0, sizeof(double) * ndof);

    const int BATCH = 4096;
    double* KeB = malloc(sizeof(double) * 900 * BATCH);
    double* MeB = malloc(sizeof(double) * 900 * BATCH);

    res->setup_seconds = wall_seconds() - t_start;
    for (int n = 1; n <= pr->n_steps; ++n) {
        /* incident velocity by the trapezoid rule */
        const double* an = pr->input_acc + 3L * (n - 1);
        for (int c = 0; c < 3; ++c) {
            vI[c] += 0.5 * dt * (aprev[c] + an[c]);
            aprev[c] = an[c];
        }

        /* UpdateCRS: K^n from D^{n-1}, C^n from h^{n-1} (Alg. 1; Eq. 1) */
        memset(Kg, 0, nb * sizeof(double));
        memcpy(Cg, Cabs, nb * sizeof(double));
        for (long e0 = 0; e0 < ne; e0 += BATCH) {
            long e1 = e0 + BATCH < ne ? e0 + BATCH : ne;
#pragma omp parallel for schedule(static)
            for (long e = e0; e < e1; ++e)
                or_element_matrices(Xall + 12 * e, D + 144 * e, pr->rho[m->layer[e]], KeB + 900 * (e - e0),
                                    MeB + 900 * (e - e0));
            for (long e = e0; e < e1; ++e) {
                double h = pr->damping_mode == 0 ? he[e] : (pr->damping_mode == 1 ? pr->h0 : 0.0);
                scatter(&P, Kg, conn + 10 * e, 10, KeB + 900 * (e - e0), 1.0);
                if (h != 0.0) {
                    scatter(&P, Cg, conn + 10 * e, 10, MeB + 900 * (e - e0), ahat * h);
                    scatter(&P, Cg, conn + 10 * e, 10, KeB + 900 * (e - e0), bhat * h);
                }
            }
        }
        for (size_t k = 0; k < nb; ++k) Ag[k] = 4.0 / (dt * dt) * Mg[k] + 2.0 / dt * Cg[k] + Kg[k];

        /* RHS of Eq. 1: f - q + C v + M (a + 4/dt v), f = 2 C_base v_I */
        spmv(&P, Cg, v, t1);
        for (long i = 0; i < ndof; ++i) t2[i] = acc[i] + 4.0 / dt * v[i];
        spmv(&P, Mg, t2, b);
        for (long i = 0; i < ndof; ++i) b[i] += t1[i] - q[i];
        for (long i = 0; i < nn; ++i) {
            const double* W = Wbase + 9 * i;
            for (int c = 0; c < 3; ++c) b[3 * i + c] += 2.0 * (W[3 * c] * vI[0] + W[3 * c + 1] * vI[1] + W[3 * c + 2] * vI[2]);
        }

        /* CRS-PCG, initial guess the previous increment */
        int its = 0;
        if (pcg(&P, Ag, b, du, pr->cg_tol, pr->cg_maxit, &its) != 0) {
            rc = fail(OR_ENOCONV, "CG did not converge", n);
            if (res->iters) res->iters[n - 1] = its;
            break;
        }
        if (res->iters) res->iters[n - 1] = its;

        /* state updates (Section 2.1) */
        spmv(&P, Kg, du, t1);
        for (long i = 0; i < ndof; ++i) {
            q[i] += t1[i];
            u[i] += du[i];
            double vn = -v[i] + 2.0 / dt * du[i];
            acc[i] = -acc[i] - 4.0 / dt * v[i] + 4.0 / (dt * dt) * du[i];
            v[i] = vn;
        }

        /* Multispring: D^n, theta^n, h^n from du^n (Alg. 1) */
        long c_rs = 0, c_rb = 0, c_rj = 0, c_cl = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : c_rs, c_rb, c_rj, c_cl)
        for (long e = 0; e < ne; ++e) {
            int l = m->layer[e];
            if (!pr->nonlinear[l]) {
                he[e] = 0.0;
                continue;
            }
            double due[30];
            for (int a = 0; a < 10; ++a)
                for (int c = 0; c < 3; ++c) due[3 * a + c] = du[3L * conn[10 * e + a] + c];
            double hsum = 0.0;
            for (int j = 0; j < 4; ++j) {
                double L[4], G[10][3], B[6][30], de[6];
                ip_bary(j, L);
                shape_grads(L, gLall + 12 * e, G);
                bmatrix(G, B);
                for (int r = 0; r < 6; ++r) {
                    double s = 0.0;
                    for (int k = 0; k < 30; ++k) s += B[r][k] * due[k];
                    de[r] = s;
                }
                double hm;
                long cnt[4] = {0, 0, 0, 0};
                ip_law(de, th + (long)sw * ns * (4 * e + j), ns, depth, pr->dirs, pr->weights, G0[l], Kb[l],
                       pr->gamma_ref[l], pr->h_max[l], D + 36 * (4 * e + j), &hm, cnt);
                c_rs += cnt[0];
                c_rb += cnt[1];
                c_rj += cnt[2];
                c_cl += cnt[3];
                hsum += hm;
            }
            he[e] = 0.25 * hsum;
        }
        res->law_events[0] += c_rs;
        res->law_events[1] += c_rb;
        res->law_events[2] += c_rj;
        res->law_events[3] += c_cl;

        for (int r = 0; r < m->n_recv; ++r) {
            int nd = m->alias ? m->alias[m->recv[r]] : m->recv[r];
            for (int c = 0; c < 3; ++c) res->vel[3L * (m->n_recv * (long)(n - 1) + r) + c] = v[3L * nd + c];
            if (res->vmax) { /* largest velocity norm over the run (surface maps of Section 3) */
                const double* vr = v + 3L * nd;
                double nv = sqrt(vr[0] * vr[0] + vr[1] * vr[1] + vr[2] * vr[2]);
                if (nv > res->vmax[r]) res->vmax[r] = nv;
            }
        }
        if (res->du_hist) memcpy(res->du_hist + ndof * (n - 1), du, sizeof(double) * ndof);
        res->steps_done = n;
    }

    if (res->u_final) memcpy(res->u_final, u, sizeof(double) * ndof);
    if (res->v_final) memcpy(res->v_final, v, sizeof(double) * ndof);
    if (res->D_final)
        for (long i = 0; i < 4L * ne; ++i) {
            int k = 0;
            for (int r = 0; r < 6; ++r)
                for (int c = r; c < 6; ++c) res->D_final[21 * i + k++] = D[36 * i + 6 * r + c];
        }
    if (res->h_final) memcpy(res->h_final, he, sizeof(double) * ne);
    if (res->theta_final) memcpy(res->theta_final, th, sizeof(double) * sw * (size_t)ne * 4 * ns);

    free(KeB); free(MeB);
    free(u); free(v); free(acc); free(q); free(du); free(b); free(t1); free(t2);
    free(D); free(th); free(he); free(Wbase);
    free(Mg); free(Kg); free(Cg); free(Cabs); free(Ag);
    free(P.rowptr); free(P.col);
    free(G0); free(Kb); free(vp);
    free(conn); free(gLall); free(vol); free(Xall);
    return rc;
}
