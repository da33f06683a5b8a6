/*
 * Plain FP64 CPU oracle for the collocation boundary element method of
 * M. J. Carley, "BEM3D: a free adaptive fast multipole boundary element
 * library" (arXiv 0908.0673).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file; only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, table or header with the GPU
 * library: every rule, constant and recursion here is written out from the
 * paper (and from the textbook definitions it cites) for this file alone.
 *
 * Everything is double precision (complex double for values) and is kept
 * plain: per-pair loops, no blocking, no reordering beyond what the
 * definitions state.  Build with -O2 -ffp-contract=off, no fast-math.
 *
 * Contents, each with the passage it follows:
 *   - 6-node isoparametric triangle and the 3-node flat
 *     triangle (every element routine takes nn = 6 or 3)     (Section 2.2)
 *   - sharp-edge DOF indexing                                 (Section 2.3)
 *   - quadrature: 7-point degree-5 rule, Duffy singular rule,
 *     uniform-subdivision near-singular rule                  (Section 2.1)
 *   - collocation matrices S, K and the free term            (Eqs. 1-3)
 *   - octree, convergence radii, near/interaction lists      (Sections 3.1, 3.4, 3.6; Eqs. 13, 14)
 *   - Taylor moments, shifts, local expansions               (Section 3.2; Eqs. 6-11)
 *   - derivatives of the Green's functions                   (Section 3.3; Eq. 12)
 *   - the fast matrix product, uniform or level-dependent
 *     expansion order                                         (Section 3.6)
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define OR_LAPLACE 0
#define OR_HELMHOLTZ 1
#define OR_R2 2 /* test-only smooth kernel G(r) = |r|^2: its Taylor series is exact */

#define OP_S 0      /* y = S x */
#define OP_K 1      /* y = K x */
#define OP_A 2      /* y = c.x - K x */
#define OP_RHS 3    /* y = -S x */
#define OP_S_REG 4  /* S with the 7-point rule on every pair, no free term */
#define OP_K_REG 5  /* K with the 7-point rule on every pair, no free term */

#define PI 3.14159265358979323846

/* ------------------------------------------------------------------ */
/* Section 2.2: the 6-node quadratic triangle on {s,t >= 0, s+t <= 1}.  */
/* Nodes: corners (0,0),(1,0),(0,1), then mid-sides of 0-1, 1-2, 2-0.  */
/* ------------------------------------------------------------------ */
static void shape6(double s, double t, double L[6], double Ls[6], double Lt[6])
{
    double z = 1.0 - s - t;
    L[0] = z * (2.0 * z - 1.0);
    L[1] = s * (2.0 * s - 1.0);
    L[2] = t * (2.0 * t - 1.0);
    L[3] = 4.0 * z * s;
    L[4] = 4.0 * s * t;
    L[5] = 4.0 * t * z;
    if (Ls) {
        Ls[0] = 1.0 - 4.0 * z; Lt[0] = 1.0 - 4.0 * z;
        Ls[1] = 4.0 * s - 1.0; Lt[1] = 0.0;
        Ls[2] = 0.0;           Lt[2] = 4.0 * t - 1.0;
        Ls[3] = 4.0 * (z - s); Lt[3] = -4.0 * s;
        Ls[4] = 4.0 * t;       Lt[4] = 4.0 * s;
        Ls[5] = -4.0 * t;      Lt[5] = 4.0 * (z - t);
    }
}

/* The first-order (3-node) triangle of Section 2.2: a flat triangle with   */
/* the linear shape functions 1 - s - t, s, t on the corners.               */
static void shape3(double s, double t, double L[6], double Ls[6], double Lt[6])
{
    for (int a = 0; a < 6; a++) L[a] = 0.0;
    L[0] = 1.0 - s - t;
    L[1] = s;
    L[2] = t;
    if (Ls) {
        for (int a = 0; a < 6; a++) Ls[a] = Lt[a] = 0.0;
        Ls[0] = -1.0; Lt[0] = -1.0;
        Ls[1] = 1.0;
        Lt[2] = 1.0;
    }
}

/* Shape functions of an element of nn nodes (3 or 6); unused entries 0. */
static void shape(int nn, double s, double t, double L[6], double Ls[6], double Lt[6])
{
    if (nn == 3) shape3(s, t, L, Ls, Lt);
    else shape6(s, t, L, Ls, Lt);
}

static const double NODE_ST[6][2] = {
    {0.0, 0.0}, {1.0, 0.0}, {0.0, 1.0}, {0.5, 0.0}, {0.5, 0.5}, {0.0, 0.5}};

/* Position, unit normal and area Jacobian of an element of nn nodes at   */
/* (s,t); L receives the shape functions (which also interpolate the     */
/* unknowns: the elements are isoparametric).                             */
static void elem_point(int nn, const double X[6][3], double s, double t, double y[3],
                       double n[3], double *J, double L[6])
{
    double Ls[6], Lt[6], ys[3] = {0, 0, 0}, yt[3] = {0, 0, 0};
    shape(nn, s, t, L, Ls, Lt);
    for (int d = 0; d < 3; d++) {
        y[d] = 0.0;
        for (int a = 0; a < nn; a++) {
            y[d] += L[a] * X[a][d];
            ys[d] += Ls[a] * X[a][d];
            yt[d] += Lt[a] * X[a][d];
        }
    }
    double N[3] = {ys[1] * yt[2] - ys[2] * yt[1], ys[2] * yt[0] - ys[0] * yt[2],
                   ys[0] * yt[1] - ys[1] * yt[0]};
    double j = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
    *J = j;
    for (int d = 0; d < 3; d++) n[d] = N[d] / j;
}

static void load_elem(int nn, const double *xyz, const int32_t *en, double X[6][3])
{
    for (int a = 0; a < 6; a++)
        for (int d = 0; d < 3; d++) X[a][d] = a < nn ? xyz[3 * (int64_t)en[a] + d] : 0.0;
}

/* Exported for tests: shape functions and the element map at (s,t). */
void or_shape(int nn, double s, double t, double *L, double *Ls, double *Lt) { shape(nn, s, t, L, Ls, Lt); }

void or_elem_point(int nn, const double *X, double s, double t, double *y, double *n, double *J)
{
    double Xe[6][3], L[6];
    for (int a = 0; a < 6; a++)
        for (int d = 0; d < 3; d++) Xe[a][d] = a < nn ? X[3 * a + d] : 0.0;
    elem_point(nn, Xe, s, t, y, n, J, L);
}

/* ------------------------------------------------------------------ */
/* Section 2.3: sharp-edge indexing.  Elements are visited in order; a */
/* node met for the first time has the normals of every element that   */
/* holds it compared with a reference normal; normals within the       */
/* tolerance share one index, a normal outside it starts a new index.  */
/* Reading: greedy clusters in element-visit order, each cluster's     */
/* reference being its first member's normal; a DOF's normal is the    */
/* normalised sum of its cluster's element normals.                    */
/* ------------------------------------------------------------------ */
int or_index_dofs(const double *xyz, int64_t n_nodes, const int32_t *elem, int64_t n_el, int nn,
                  double tol_deg, int32_t *elem_dofs, int32_t *dof_node, double *dof_normal,
                  int64_t *n_dof_out)
{
    int64_t *cnt = calloc(n_nodes + 1, sizeof *cnt);
    for (int64_t e = 0; e < n_el; e++)
        for (int a = 0; a < nn; a++) {
            int32_t g = elem[nn * e + a];
            if (g < 0 || g >= n_nodes) { free(cnt); return -1; }
            cnt[g + 1]++;
        }
    for (int64_t g = 0; g < n_nodes; g++) cnt[g + 1] += cnt[g];
    int64_t *fill = malloc((n_nodes + 1) * sizeof *fill);
    memcpy(fill, cnt, (n_nodes + 1) * sizeof *fill);
    int64_t *inc = malloc(nn * n_el * sizeof *inc); /* incidence = nn*e + a, in element order */
    for (int64_t e = 0; e < n_el; e++)
        for (int a = 0; a < nn; a++) inc[fill[elem[nn * e + a]]++] = nn * e + a;
    for (int64_t i = 0; i < nn * n_el; i++) elem_dofs[i] = -1;

    double cos_tol = cos(tol_deg * PI / 180.0);
    int64_t n_dof = 0;
    double (*nrm)[3] = malloc(nn * n_el * sizeof *nrm);
    int64_t *ref = malloc(nn * n_el * sizeof *ref);
    for (int64_t e = 0; e < n_el; e++) {
        for (int a = 0; a < nn; a++) {
            if (elem_dofs[nn * e + a] >= 0) continue;
            int32_t g = elem[nn * e + a];
            int64_t first_dof = n_dof;
            for (int64_t p = cnt[g]; p < cnt[g + 1]; p++) {
                int64_t e2 = inc[p] / nn;
                int a2 = (int)(inc[p] % nn);
                double X[6][3], y[3], n[3], J, L[6];
                load_elem(nn, xyz, elem + nn * e2, X);
                elem_point(nn, X, NODE_ST[a2][0], NODE_ST[a2][1], y, n, &J, L);
                int64_t hit = -1;
                for (int64_t c = first_dof; c < n_dof; c++) {
                    const double *r = nrm[ref[c]];
                    if (n[0] * r[0] + n[1] * r[1] + n[2] * r[2] > cos_tol) { hit = c; break; }
                }
                memcpy(nrm[p], n, sizeof n);
                if (hit < 0) {
                    hit = n_dof++;
                    ref[hit] = p;
                    dof_node[hit] = g;
                    dof_normal[3 * hit] = dof_normal[3 * hit + 1] = dof_normal[3 * hit + 2] = 0.0;
                }
                elem_dofs[nn * e2 + a2] = (int32_t)hit;
                for (int d = 0; d < 3; d++) dof_normal[3 * hit + d] += n[d];
            }
        }
    }
    for (int64_t i = 0; i < n_dof; i++) {
        double *v = dof_normal + 3 * i;
        double l = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        for (int d = 0; d < 3; d++) v[d] /= l;
    }
    *n_dof_out = n_dof;
    free(cnt); free(fill); free(inc); free(nrm); free(ref);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Quadrature rules on the reference triangle (weights sum to 1/2).    */
/* ------------------------------------------------------------------ */
#define MAXQ 1792 /* 4^4 sub-triangles x 7 points */

typedef struct { int n; double s[MAXQ], t[MAXQ], w[MAXQ]; } rule_t;

/* Radon's 7-point degree-5 rule (Stroud T2:5-1), barycentric form. */
static void rule7_bary(double b[7][3], double w[7])
{
    double r15 = sqrt(15.0);
    double a = (6.0 - r15) / 21.0, c = (6.0 + r15) / 21.0;
    double wa = (155.0 - r15) / 1200.0, wc = (155.0 + r15) / 1200.0;
    double t[7][3] = {{1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0},
                      {a, a, 1.0 - 2.0 * a}, {a, 1.0 - 2.0 * a, a}, {1.0 - 2.0 * a, a, a},
                      {c, c, 1.0 - 2.0 * c}, {c, 1.0 - 2.0 * c, c}, {1.0 - 2.0 * c, c, c}};
    double ww[7] = {9.0 / 40.0, wa, wa, wa, wc, wc, wc};
    memcpy(b, t, sizeof t);
    memcpy(w, ww, sizeof ww);
}

/* 7-point rule mapped onto the sub-triangle (A,B,C) of the reference triangle. */
static void add_rule7(rule_t *r, const double A[2], const double B[2], const double C[2])
{
    double b[7][3], w[7];
    rule7_bary(b, w);
    double area = 0.5 * fabs((B[0] - A[0]) * (C[1] - A[1]) - (C[0] - A[0]) * (B[1] - A[1]));
    for (int q = 0; q < 7; q++) {
        r->s[r->n] = b[q][0] * A[0] + b[q][1] * B[0] + b[q][2] * C[0];
        r->t[r->n] = b[q][0] * A[1] + b[q][1] * B[1] + b[q][2] * C[1];
        r->w[r->n] = w[q] * area;
        r->n++;
    }
}

static void rule_regular(rule_t *r)
{
    static const double A[2] = {0, 0}, B[2] = {1, 0}, C[2] = {0, 1};
    r->n = 0;
    add_rule7(r, A, B, C);
}

static void subdiv(rule_t *r, const double A[2], const double B[2], const double C[2], int d)
{
    if (d == 0) { add_rule7(r, A, B, C); return; }
    double ab[2] = {0.5 * (A[0] + B[0]), 0.5 * (A[1] + B[1])};
    double bc[2] = {0.5 * (B[0] + C[0]), 0.5 * (B[1] + C[1])};
    double ca[2] = {0.5 * (C[0] + A[0]), 0.5 * (C[1] + A[1])};
    subdiv(r, A, ab, ca, d - 1);
    subdiv(r, ab, B, bc, d - 1);
    subdiv(r, ca, bc, C, d - 1);
    subdiv(r, ab, bc, ca, d - 1);
}

/* Near-singular rule: 4^d congruent sub-triangles, 7 points each. */
static void rule_subdiv(rule_t *r, int d)
{
    static const double A[2] = {0, 0}, B[2] = {1, 0}, C[2] = {0, 1};
    r->n = 0;
    subdiv(r, A, B, C, d);
}

/* Gauss-Legendre nodes and weights on [0,1] by Newton's method on P_n. */
static void gauss_legendre01(int n, double *x, double *w)
{
    for (int i = 0; i < n; i++) {
        double z = cos(PI * (i + 0.75) / (n + 0.5)), dp = 0.0;
        for (int it = 0; it < 100; it++) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; k++) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; k++) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
        }
        x[i] = 0.5 * (1.0 - z);
        w[i] = 1.0 / ((1.0 - z * z) * dp * dp);
    }
}

/* Duffy rule for a sub-triangle (P,A,B) with the singular point at P:
 * (u,v) in [0,1]^2 -> P + u (A - P) + u v (B - A), Jacobian u |det|.     */
static void add_duffy(rule_t *r, const double P[2], const double A[2], const double B[2], int ng)
{
    double x[32], w[32];
    gauss_legendre01(ng, x, w);
    double det = fabs((A[0] - P[0]) * (B[1] - A[1]) - (A[1] - P[1]) * (B[0] - A[0]));
    for (int i = 0; i < ng; i++)
        for (int j = 0; j < ng; j++) {
            double u = x[i], v = x[j];
            r->s[r->n] = P[0] + u * (A[0] - P[0]) + u * v * (B[0] - A[0]);
            r->t[r->n] = P[1] + u * (A[1] - P[1]) + u * v * (B[1] - A[1]);
            r->w[r->n] = w[i] * w[j] * u * det;
            r->n++;
        }
}

/* Singular rule about element node a: one Duffy triangle for a corner,
 * two for a mid-side node.                                                */
static void rule_singular(rule_t *r, int a, int ng)
{
    static const double V[3][2] = {{0, 0}, {1, 0}, {0, 1}};
    r->n = 0;
    if (a < 3) {
        add_duffy(r, V[a], V[(a + 1) % 3], V[(a + 2) % 3], ng);
    } else {
        int c0 = a - 3, c1 = (a - 2) % 3, c2 = (a - 1) % 3; /* mid-side of c0-c1; opposite corner c2 */
        add_duffy(r, NODE_ST[a], V[c1], V[c2], ng);
        add_duffy(r, NODE_ST[a], V[c2], V[c0], ng);
    }
}

/* Exported for tests: the rules' points. kind 0 regular, 1 subdivision(d=param),
 * 2 singular(node=param).  Returns the point count.                      */
int or_rule(int kind, int param, int ng, double *s, double *t, double *w)
{
    static rule_t r;
    if (kind == 0) rule_regular(&r);
    else if (kind == 1) rule_subdiv(&r, param);
    else rule_singular(&r, param, ng);
    memcpy(s, r.s, r.n * sizeof(double));
    memcpy(t, r.t, r.n * sizeof(double));
    memcpy(w, r.w, r.n * sizeof(double));
    return r.n;
}

/* ------------------------------------------------------------------ */
/* Green's functions (Eqs. 1a/b) and their normal derivative at the    */
/* source point, d/dn1 G(|x - y|) = n1 . grad_y G.                     */
/* ------------------------------------------------------------------ */
static void kernel(int green, double k, const double x[3], const double y[3], const double n[3],
                   cplx *G, cplx *dG)
{
    double r[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
    double R2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    double rn = r[0] * n[0] + r[1] * n[1] + r[2] * n[2];
    if (green == OR_R2) {
        *G = R2;
        *dG = -2.0 * rn;
        return;
    }
    double R = sqrt(R2);
    if (green == OR_LAPLACE) {
        *G = 1.0 / (4.0 * PI * R);
        *dG = rn / (4.0 * PI * R * R2);
    } else {
        cplx e = cexp(I * k * R);
        *G = e / (4.0 * PI * R);
        *dG = (1.0 - I * k * R) * e * rn / (4.0 * PI * R * R2);
    }
}

/* Integrals over one element of L_a G and L_a dG/dn1 for target x. */
static void elem_integrals(int nn, const double X[6][3], const double x[3], int green, double k,
                           const rule_t *r, cplx S[6], cplx K[6])
{
    for (int a = 0; a < 6; a++) S[a] = K[a] = 0.0;
    for (int q = 0; q < r->n; q++) {
        double y[3], n[3], J, L[6];
        cplx G, dG;
        elem_point(nn, X, r->s[q], r->t[q], y, n, &J, L);
        kernel(green, k, x, y, n, &G, &dG);
        double wj = r->w[q] * J;
        for (int a = 0; a < nn; a++) {
            S[a] += wj * L[a] * G;
            K[a] += wj * L[a] * dG;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Pair classification (the paper names singular and near-singular     */
/* rules without thresholds).  Reading: singular when the target's     */
/* geometric node is a node of the element; near-singular when         */
/* |x - c_m| < 2 h_m with c_m the corner mean and h_m the largest      */
/* corner-mean-to-node distance; then 4^d sub-triangles with the least */
/* d >= 1 such that h_m/2^d <= |x - c_m|/2, at most 4.                  */
/* ------------------------------------------------------------------ */
#define CL_REGULAR 0
#define CL_NEAR 1
#define CL_SINGULAR 2

static int classify(int nn, const double *xyz, const int32_t *en, int32_t tgt_node, const double x[3],
                    int *param)
{
    for (int a = 0; a < nn; a++)
        if (en[a] == tgt_node) { *param = a; return CL_SINGULAR; }
    double cm[3];
    for (int d = 0; d < 3; d++)
        cm[d] = ((xyz[3 * (int64_t)en[0] + d] + xyz[3 * (int64_t)en[1] + d]) + xyz[3 * (int64_t)en[2] + d]) / 3.0;
    double h2 = 0.0;
    for (int a = 0; a < nn; a++) {
        const double *p = xyz + 3 * (int64_t)en[a];
        double dx = p[0] - cm[0], dy = p[1] - cm[1], dz = p[2] - cm[2];
        double v = (dx * dx + dy * dy) + dz * dz;
        if (v > h2) h2 = v;
    }
    double dx = x[0] - cm[0], dy = x[1] - cm[1], dz = x[2] - cm[2];
    double d2 = (dx * dx + dy * dy) + dz * dz;
    if (!(d2 < 4.0 * h2)) return CL_REGULAR;
    int d = 1;
    double f = 4.0;
    while (d < 4 && 4.0 * h2 > d2 * f) { d++; f *= 4.0; }
    *param = d;
    return CL_NEAR;
}

int or_classify(int nn, const double *xyz, const int32_t *en, int32_t tgt_node, const double *x, int *param)
{
    *param = 0;
    return classify(nn, xyz, en, tgt_node, x, param);
}

#define NGAUSS 12

/* Accurate (S, K) integrals of one (target, element) pair, and the same
 * with the 7-point rule; kind is the classification.                     */
static int pair_integrals(int nn, const double *xyz, const int32_t *en, int32_t tgt_node, const double x[3],
                          int green, double k, cplx S[6], cplx K[6], cplx Sr[6], cplx Kr[6])
{
    double X[6][3];
    load_elem(nn, xyz, en, X);
    static __thread rule_t reg, acc;
    rule_regular(&reg);
    elem_integrals(nn, X, x, green, k, &reg, Sr, Kr);
    int param = 0, cls = green == OR_R2 ? CL_REGULAR : classify(nn, xyz, en, tgt_node, x, &param);
    if (cls == CL_REGULAR) {
        memcpy(S, Sr, 6 * sizeof(cplx));
        memcpy(K, Kr, 6 * sizeof(cplx));
        return cls;
    }
    if (cls == CL_SINGULAR) rule_singular(&acc, param, NGAUSS);
    else rule_subdiv(&acc, param);
    elem_integrals(nn, X, x, green, k, &acc, S, K);
    return cls;
}

/* Exported for tests: accurate integrals of one pair (interleaved complex). */
int or_pair(int nn, const double *xyz, const int32_t *en, int32_t tgt_node, const double *x, int green,
            double k, double *S12, double *K12)
{
    cplx S[6], K[6], Sr[6], Kr[6];
    int c = pair_integrals(nn, xyz, en, tgt_node, x, green, k, S, K, Sr, Kr);
    for (int a = 0; a < 6; a++) {
        S12[2 * a] = creal(S[a]); S12[2 * a + 1] = cimag(S[a]);
        K12[2 * a] = creal(K[a]); K12[2 * a + 1] = cimag(K[a]);
    }
    return c;
}

/* ------------------------------------------------------------------ */
/* Eq. 3: collocation matrices.  Reading of the signs: n points out of */
/* the body; the equation solved is c_i phi_i - sum_j K_ij phi_j =     */
/* - sum_j S_ij chi_j with c_i = 1 + sum_j K0_ij (Eq. 2, G0 = 1/4piR). */
/* ------------------------------------------------------------------ */
typedef struct {
    const double *xyz;
    const int32_t *elem, *elem_dofs, *dof_node; /* elem, elem_dofs: [n_el][nn] */
    int64_t n_el, n_dof;
    int nn; /* nodes per element: 3 (first order) or 6 (second order) */
} mesh_t;

/* One row: S_i., K_i. (dense, length n_dof) and the free term c_i. */
static void assemble_row(const mesh_t *m, int64_t i, int green, double k, int regular_only,
                         cplx *Srow, cplx *Krow, double *c)
{
    const double *x = m->xyz + 3 * (int64_t)m->dof_node[i];
    double k0sum = 0.0;
    for (int64_t e = 0; e < m->n_el; e++) {
        const int32_t *en = m->elem + m->nn * e;
        cplx S[6], K[6], Sr[6], Kr[6];
        int cls = pair_integrals(m->nn, m->xyz, en, m->dof_node[i], x, green, k, S, K, Sr, Kr);
        if (regular_only) { memcpy(S, Sr, sizeof S); memcpy(K, Kr, sizeof K); }
        for (int a = 0; a < m->nn; a++) {
            int32_t j = m->elem_dofs[m->nn * e + a];
            if (Srow) Srow[j] += S[a];
            if (Krow) Krow[j] += K[a];
        }
        if (c) {
            cplx S0[6], K0[6];
            if (green == OR_LAPLACE) memcpy(K0, K, sizeof K0);
            else if (cls == CL_REGULAR) {
                double X[6][3];
                rule_t reg;
                load_elem(m->nn, m->xyz, en, X);
                rule_regular(&reg);
                elem_integrals(m->nn, X, x, OR_LAPLACE, 0.0, &reg, S0, K0);
            } else {
                cplx a1[6], a2[6];
                pair_integrals(m->nn, m->xyz, en, m->dof_node[i], x, OR_LAPLACE, 0.0, S0, K0, a1, a2);
            }
            for (int a = 0; a < m->nn; a++) k0sum += creal(K0[a]);
        }
    }
    if (c) *c = 1.0 + k0sum;
}

/* Dense S, K (row-major n x n, interleaved complex) and free term c. */
int or_assemble(const double *xyz, const int32_t *elem, const int32_t *elem_dofs,
                const int32_t *dof_node, int64_t n_el, int64_t n_dof, int nn, int green, double k,
                double *S, double *K, double *c)
{
    mesh_t m = {xyz, elem, elem_dofs, dof_node, n_el, n_dof, nn};
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < n_dof; i++) {
        cplx *Sr = (cplx *)S + i * n_dof, *Kr = (cplx *)K + i * n_dof;
        for (int64_t j = 0; j < n_dof; j++) Sr[j] = Kr[j] = 0.0;
        assemble_row(&m, i, green, k, 0, Sr, Kr, c + i);
    }
    return 0;
}

/* Direct matrix-vector product on selected rows.  x, y interleaved complex. */
int or_matvec_rows(const double *xyz, const int32_t *elem, const int32_t *elem_dofs,
                   const int32_t *dof_node, int64_t n_el, int64_t n_dof, int nn, int green, double k,
                   int op, const double *x, const int64_t *rows, int64_t nrows, double *y)
{
    mesh_t m = {xyz, elem, elem_dofs, dof_node, n_el, n_dof, nn};
    const cplx *xc = (const cplx *)x;
    cplx *yc = (cplx *)y;
    int regular = (op == OP_S_REG || op == OP_K_REG);
    int use_S = (op == OP_S || op == OP_RHS || op == OP_S_REG);
#pragma omp parallel
    {
        cplx *row = malloc(n_dof * sizeof(cplx));
#pragma omp for schedule(dynamic, 4)
        for (int64_t r = 0; r < nrows; r++) {
            int64_t i = rows[r];
            for (int64_t j = 0; j < n_dof; j++) row[j] = 0.0;
            double c = 0.0;
            assemble_row(&m, i, green, k, regular, use_S ? row : NULL, use_S ? NULL : row,
                         op == OP_A ? &c : NULL);
            cplx acc = 0.0;
            for (int64_t j = 0; j < n_dof; j++) acc += row[j] * xc[j];
            if (op == OP_A) yc[r] = c * xc[i] - acc;
            else if (op == OP_RHS) yc[r] = -acc;
            else yc[r] = acc;
        }
        free(row);
    }
    return 0;
}

/* Free term alone on selected rows. */
int or_free_term(const double *xyz, const int32_t *elem, const int32_t *elem_dofs,
                 const int32_t *dof_node, int64_t n_el, int64_t n_dof, int nn, const int64_t *rows,
                 int64_t nrows, double *c)
{
    mesh_t m = {xyz, elem, elem_dofs, dof_node, n_el, n_dof, nn};
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t r = 0; r < nrows; r++) assemble_row(&m, rows[r], OR_LAPLACE, 0.0, 0, NULL, NULL, c + r);
    return 0;
}

/* Potential of single/double layer densities at arbitrary points (regular
 * and near-singular rules only: the points must not lie on the surface). */
int or_layer_potential(const double *xyz, const int32_t *elem, const int32_t *elem_dofs,
                       int64_t n_el, int nn, int green, double k, const double *sig_s,
                       const double *sig_d, const double *pts, int64_t npts, double *out)
{
    const cplx *ss = (const cplx *)sig_s, *sd = (const cplx *)sig_d;
    cplx *o = (cplx *)out;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t p = 0; p < npts; p++) {
        cplx acc = 0.0;
        for (int64_t e = 0; e < n_el; e++) {
            cplx S[6], K[6], Sr[6], Kr[6];
            pair_integrals(nn, xyz, elem + nn * e, -1, pts + 3 * p, green, k, S, K, Sr, Kr);
            for (int a = 0; a < nn; a++) {
                int32_t j = elem_dofs[nn * e + a];
                if (ss) acc += S[a] * ss[j];
                if (sd) acc += K[a] * sd[j];
            }
        }
        o[p] = acc;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Sections 3.1, 3.4, 3.6: the octree.                                 */
/* Readings: each element is keyed by the mean of its corners and owned */
/* by exactly one leaf; targets are the DOF positions; a box exists    */
/* when it holds an element key or a target; it is split when it holds */
/* more than B elements and is above level 21.  The root is a cube     */
/* padded by 2^-20 of its side around all nodes.  Keys quantise each   */
/* coordinate to 21 bits and interleave them (x highest in each        */
/* triplet).  Boxes are ordered by (level, key prefix).                */
/* ------------------------------------------------------------------ */
#define MAXLEV 21

typedef struct {
    int level, leaf, parent, child_begin, nchild;
    uint64_t prefix;
    int64_t eb, ee, tb, te; /* ranges in the sorted element / target orders */
    double c[3], r;
} obox_t;

typedef struct {
    int64_t n_box, n_el, n_tgt;
    obox_t *box;
    int64_t *eperm, *tperm;
    uint64_t *ekey, *tkey; /* sorted keys */
    int64_t *near_ptr, *near_idx, *inter_ptr, *inter_idx;
    double corner[3], side;
    int max_level;
    int literal; /* sources are the DOFs (node basis functions); eb/ee = tb/te */
} otree_t;

static uint64_t spread3(uint64_t v)
{
    uint64_t r = 0;
    for (int b = 0; b < 21; b++) r |= ((v >> b) & 1u) << (3 * b);
    return r;
}

static uint64_t compact3(uint64_t v)
{
    uint64_t r = 0;
    for (int b = 0; b < 21; b++) r |= ((v >> (3 * b)) & 1u) << b;
    return r;
}

static uint64_t morton(const double p[3], const double corner[3], double scale)
{
    uint64_t q[3];
    for (int d = 0; d < 3; d++) {
        double v = floor((p[d] - corner[d]) * scale);
        if (v < 0.0) v = 0.0;
        if (v > 2097151.0) v = 2097151.0;
        q[d] = (uint64_t)v;
    }
    return (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
}

typedef struct { uint64_t key; int64_t id; } kv_t;

static int cmp_kv(const void *a, const void *b)
{
    const kv_t *x = a, *y = b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->id < y->id ? -1 : (x->id > y->id);
}

static int64_t lower_bound(const uint64_t *a, int64_t n, uint64_t v)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (a[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

static double dist3(const double a[3], const double b[3])
{
    double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return sqrt((dx * dx + dy * dy) + dz * dz);
}

typedef struct { obox_t *v; int64_t n, cap; } boxvec_t;

static void push_box(boxvec_t *bv, obox_t b)
{
    if (bv->n == bv->cap) {
        bv->cap = bv->cap ? 2 * bv->cap : 1024;
        bv->v = realloc(bv->v, bv->cap * sizeof(obox_t));
    }
    bv->v[bv->n++] = b;
}

/* Recursive subdivision over prefix ranges of the sorted keys. */
static void build_rec(otree_t *T, boxvec_t *bv, int level, uint64_t prefix, int B, int max_depth)
{
    int shift = 3 * (MAXLEV - level);
    uint64_t lo = prefix << shift;
    uint64_t hi_excl_known = (level == 0);
    obox_t b;
    memset(&b, 0, sizeof b);
    b.level = level;
    b.prefix = prefix;
    b.eb = lower_bound(T->ekey, T->n_el, lo);
    b.tb = lower_bound(T->tkey, T->n_tgt, lo);
    if (level == 0) { b.ee = T->n_el; b.te = T->n_tgt; }
    else {
        uint64_t hi = (prefix + 1) << shift;
        b.ee = lower_bound(T->ekey, T->n_el, hi);
        b.te = lower_bound(T->tkey, T->n_tgt, hi);
    }
    (void)hi_excl_known;
    if (b.ee - b.eb == 0 && b.te - b.tb == 0) return;
    b.leaf = !((b.ee - b.eb) > B && level < max_depth);
    push_box(bv, b);
    if (!b.leaf)
        for (uint64_t c = 0; c < 8; c++) build_rec(T, bv, level + 1, (prefix << 3) | c, B, max_depth);
}

static int cmp_box(const void *a, const void *b)
{
    const obox_t *x = a, *y = b;
    if (x->level != y->level) return x->level - y->level;
    return x->prefix < y->prefix ? -1 : (x->prefix > y->prefix);
}

static int64_t find_box(const otree_t *T, const int64_t *lev_off, int level, uint64_t prefix)
{
    int64_t lo = lev_off[level], hi = lev_off[level + 1];
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (T->box[mid].prefix < prefix) lo = mid + 1; else hi = mid;
    }
    return lo;
}

static int sep(const obox_t *X, const obox_t *Y, double theta, double kappa, double k)
{
    double s = X->r + Y->r;
    if (kappa > 0.0 && isfinite(kappa) && k * s > kappa) return 0;
    return dist3(X->c, Y->c) > s / theta;
}

typedef struct { int64_t *v; int64_t n, cap; } ivec_t;

static void ipush(ivec_t *a, int64_t x)
{
    if (a->n == a->cap) {
        a->cap = a->cap ? 2 * a->cap : 16;
        a->v = realloc(a->v, a->cap * sizeof(int64_t));
    }
    a->v[a->n++] = x;
}

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return x < y ? -1 : (x > y);
}

/* attach = 1 (with tgt_node, the geometric node of each target): a leaf's */
/* radius also covers every node of every element attached to the nodes of */
/* its targets, as Section 3.6 defines r_C (the elements attached to a     */
/* leaf's vertices, Section 3.1); sources stay owned by one leaf each.     */
/* attach = 2, the paper's tree read literally (Sections 3.1, 3.6): the    */
/* boxes are built over the DOF points alone, B counts DOFs, each DOF's    */
/* basis function is a source of its box, and the radius of a leaf covers  */
/* its DOF points and every node of every element attached to them.  The   */
/* element ranges of the boxes are then their DOF ranges (eb = tb, ...).   */
void *or_tree_build(const double *xyz, int64_t n_nodes, const int32_t *elem, int64_t n_el, int nn,
                    const double *tgt_xyz, const int32_t *tgt_node, int64_t n_tgt, int B, int max_depth,
                    double theta, double kappa, double k, int attach)
{
    otree_t *T = calloc(1, sizeof *T);
    T->literal = attach == 2;
    const int64_t n_mesh_el = n_el;
    if (T->literal) n_el = n_tgt; /* the DOFs stand in the element slots of the tree */
    T->n_el = n_el;
    T->n_tgt = n_tgt;
    /* root cube */
    double lo[3], hi[3];
    for (int d = 0; d < 3; d++) { lo[d] = xyz[d]; hi[d] = xyz[d]; }
    for (int64_t i = 0; i < n_nodes; i++)
        for (int d = 0; d < 3; d++) {
            double v = xyz[3 * i + d];
            if (v < lo[d]) lo[d] = v;
            if (v > hi[d]) hi[d] = v;
        }
    double ext = 0.0;
    for (int d = 0; d < 3; d++) if (hi[d] - lo[d] > ext) ext = hi[d] - lo[d];
    T->side = ext * (1.0 + 0x1p-20);
    for (int d = 0; d < 3; d++) T->corner[d] = (lo[d] + hi[d]) * 0.5 - T->side * 0.5;
    double scale = 2097152.0 / T->side;

    /* keys, sorted by (key, id) */
    kv_t *ek = malloc((n_el > 0 ? n_el : 1) * sizeof *ek), *tk = malloc((n_tgt > 0 ? n_tgt : 1) * sizeof *tk);
    for (int64_t e = 0; e < n_el; e++) {
        double p[3];
        if (T->literal) { /* the DOF points */
            ek[e].key = morton(tgt_xyz + 3 * e, T->corner, scale);
            ek[e].id = e;
            continue;
        }
        const int32_t *en = elem + nn * e;
        for (int d = 0; d < 3; d++)
            p[d] = ((xyz[3 * (int64_t)en[0] + d] + xyz[3 * (int64_t)en[1] + d]) + xyz[3 * (int64_t)en[2] + d]) / 3.0;
        ek[e].key = morton(p, T->corner, scale);
        ek[e].id = e;
    }
    for (int64_t i = 0; i < n_tgt; i++) {
        tk[i].key = morton(tgt_xyz + 3 * i, T->corner, scale);
        tk[i].id = i;
    }
    qsort(ek, n_el, sizeof *ek, cmp_kv);
    qsort(tk, n_tgt, sizeof *tk, cmp_kv);
    T->eperm = malloc((n_el + 1) * sizeof(int64_t));
    T->tperm = malloc((n_tgt + 1) * sizeof(int64_t));
    T->ekey = malloc((n_el + 1) * sizeof(uint64_t));
    T->tkey = malloc((n_tgt + 1) * sizeof(uint64_t));
    for (int64_t e = 0; e < n_el; e++) { T->eperm[e] = ek[e].id; T->ekey[e] = ek[e].key; }
    for (int64_t i = 0; i < n_tgt; i++) { T->tperm[i] = tk[i].id; T->tkey[i] = tk[i].key; }
    free(ek); free(tk);

    boxvec_t bv = {0};
    build_rec(T, &bv, 0, 0, B, max_depth);
    qsort(bv.v, bv.n, sizeof(obox_t), cmp_box);
    T->box = bv.v;
    T->n_box = bv.n;
    int64_t lev_off[MAXLEV + 3] = {0};
    for (int64_t b = 0; b < T->n_box; b++) lev_off[T->box[b].level + 1]++;
    for (int l = 0; l <= MAXLEV + 1; l++) lev_off[l + 1] += lev_off[l];
    T->max_level = 0;
    for (int64_t b = 0; b < T->n_box; b++) if (T->box[b].level > T->max_level) T->max_level = T->box[b].level;

    /* topology, centres */
    for (int64_t b = 0; b < T->n_box; b++) {
        obox_t *x = &T->box[b];
        x->parent = x->level ? (int)find_box(T, lev_off, x->level - 1, x->prefix >> 3) : -1;
        x->child_begin = -1;
        x->nchild = 0;
        double h = ldexp(T->side, -x->level);
        uint64_t ip[3] = {compact3(x->prefix >> 2), compact3(x->prefix >> 1), compact3(x->prefix)};
        for (int d = 0; d < 3; d++) x->c[d] = T->corner[d] + h * ((double)ip[d] + 0.5);
    }
    for (int64_t b = 0; b < T->n_box; b++) {
        obox_t *x = &T->box[b];
        if (x->parent >= 0) {
            obox_t *p = &T->box[x->parent];
            if (p->child_begin < 0) p->child_begin = (int)b;
            p->nchild++;
        }
    }
    /* elements holding each node (attach mode) */
    int64_t *ns = NULL, *ne_of = NULL;
    if (attach) {
        ns = calloc(n_nodes + 1, sizeof *ns);
        for (int64_t i = 0; i < nn * n_mesh_el; i++) ns[elem[i] + 1]++;
        for (int64_t g = 0; g < n_nodes; g++) ns[g + 1] += ns[g];
        int64_t *fill = malloc((n_nodes + 1) * sizeof *fill);
        memcpy(fill, ns, (n_nodes + 1) * sizeof *fill);
        ne_of = malloc((nn * n_mesh_el + 1) * sizeof *ne_of);
        for (int64_t i = 0; i < nn * n_mesh_el; i++) ne_of[fill[elem[i]]++] = i / nn;
        free(fill);
    }
    /* Section 3.4: convergence radii.  Leaf: farthest node of an owned
     * element or owned target from the centre (and, attach mode, of an
     * element attached to a target's node).  Parent: Eq. 13.             */
    double sqrt3 = sqrt(3.0);
    for (int64_t b = T->n_box - 1; b >= 0; b--) {
        obox_t *x = &T->box[b];
        double r = 0.0;
        if (x->leaf) {
            for (int64_t e = x->eb; e < x->ee && !T->literal; e++)
                for (int a = 0; a < nn; a++) {
                    double v = dist3(xyz + 3 * (int64_t)elem[nn * T->eperm[e] + a], x->c);
                    if (v > r) r = v;
                }
            for (int64_t i = x->tb; i < x->te; i++) {
                double v = dist3(tgt_xyz + 3 * T->tperm[i], x->c);
                if (v > r) r = v;
                if (!attach) continue;
                int32_t g = tgt_node[T->tperm[i]];
                for (int64_t p = ns[g]; p < ns[g + 1]; p++)
                    for (int a = 0; a < nn; a++) {
                        double w = dist3(xyz + 3 * (int64_t)elem[nn * ne_of[p] + a], x->c);
                        if (w > r) r = w;
                    }
            }
        } else {
            double rc = 0.0;
            for (int c = 0; c < x->nchild; c++)
                if (T->box[x->child_begin + c].r > rc) rc = T->box[x->child_begin + c].r;
            double hc = ldexp(T->side, -(x->level + 1));
            r = rc + (sqrt3 * hc) * 0.5;
        }
        x->r = r;
    }
    free(ns);
    free(ne_of);
    /* Section 3.6: near-field and interaction lists, descending the tree;
     * Eq. 14 with a safety factor theta (paper: theta = 1) and, for
     * Helmholtz, the extra bound k (r1 + r2) <= kappa (paper: none).
     * Boxes with no element below them are sources of nothing.           */
    ivec_t *nl = calloc(T->n_box, sizeof(ivec_t)), *il = calloc(T->n_box, sizeof(ivec_t));
    ipush(&nl[0], 0);
    for (int64_t b = 1; b < T->n_box; b++) {
        obox_t *B_ = &T->box[b];
        ivec_t *pn = &nl[B_->parent];
        for (int64_t j = 0; j < pn->n; j++) {
            obox_t *N = &T->box[pn->v[j]];
            if (N->leaf) {
                if (N->ee == N->eb) continue;
                if (sep(B_, N, theta, kappa, k)) ipush(&il[b], pn->v[j]);
                else ipush(&nl[b], pn->v[j]);
            } else {
                for (int c = 0; c < N->nchild; c++) {
                    int64_t ci = N->child_begin + c;
                    obox_t *C = &T->box[ci];
                    if (C->ee == C->eb) continue;
                    if (sep(B_, C, theta, kappa, k)) ipush(&il[b], ci);
                    else ipush(&nl[b], ci);
                }
            }
        }
    }
    T->near_ptr = calloc(T->n_box + 1, sizeof(int64_t));
    T->inter_ptr = calloc(T->n_box + 1, sizeof(int64_t));
    for (int64_t b = 0; b < T->n_box; b++) {
        qsort(nl[b].v, nl[b].n, sizeof(int64_t), cmp_i64);
        qsort(il[b].v, il[b].n, sizeof(int64_t), cmp_i64);
        T->near_ptr[b + 1] = T->near_ptr[b] + nl[b].n;
        T->inter_ptr[b + 1] = T->inter_ptr[b] + il[b].n;
    }
    T->near_idx = malloc((T->near_ptr[T->n_box] + 1) * sizeof(int64_t));
    T->inter_idx = malloc((T->inter_ptr[T->n_box] + 1) * sizeof(int64_t));
    for (int64_t b = 0; b < T->n_box; b++) {
        if (nl[b].n) memcpy(T->near_idx + T->near_ptr[b], nl[b].v, nl[b].n * sizeof(int64_t));
        if (il[b].n) memcpy(T->inter_idx + T->inter_ptr[b], il[b].v, il[b].n * sizeof(int64_t));
        free(nl[b].v); free(il[b].v);
    }
    free(nl); free(il);
    return T;
}

void or_tree_sizes(const void *h, int64_t *sz /* n_box, n_near, n_inter, max_level */)
{
    const otree_t *T = h;
    sz[0] = T->n_box;
    sz[1] = T->near_ptr[T->n_box];
    sz[2] = T->inter_ptr[T->n_box];
    sz[3] = T->max_level;
}

/* Export: per box int64 [n_box][10] = level, leaf, parent, child_begin, nchild,
 * eb, ee, tb, te, prefix; double [n_box][4] = centre, radius.               */
void or_tree_export(const void *h, int64_t *ibox, double *dbox, int64_t *eperm, int64_t *tperm,
                    int64_t *near_ptr, int64_t *near_idx, int64_t *inter_ptr, int64_t *inter_idx,
                    double *root /* corner[3], side */)
{
    const otree_t *T = h;
    for (int64_t b = 0; b < T->n_box; b++) {
        const obox_t *x = &T->box[b];
        int64_t *o = ibox + 10 * b;
        o[0] = x->level; o[1] = x->leaf; o[2] = x->parent; o[3] = x->child_begin; o[4] = x->nchild;
        o[5] = x->eb; o[6] = x->ee; o[7] = x->tb; o[8] = x->te; o[9] = (int64_t)x->prefix;
        for (int d = 0; d < 3; d++) dbox[4 * b + d] = x->c[d];
        dbox[4 * b + 3] = x->r;
    }
    memcpy(eperm, T->eperm, T->n_el * sizeof(int64_t));
    memcpy(tperm, T->tperm, T->n_tgt * sizeof(int64_t));
    memcpy(near_ptr, T->near_ptr, (T->n_box + 1) * sizeof(int64_t));
    memcpy(inter_ptr, T->inter_ptr, (T->n_box + 1) * sizeof(int64_t));
    memcpy(near_idx, T->near_idx, T->near_ptr[T->n_box] * sizeof(int64_t));
    memcpy(inter_idx, T->inter_idx, T->inter_ptr[T->n_box] * sizeof(int64_t));
    for (int d = 0; d < 3; d++) root[d] = T->corner[d];
    root[3] = T->side;
}

void or_tree_free(void *h)
{
    otree_t *T = h;
    if (!T) return;
    free(T->box); free(T->eperm); free(T->tperm); free(T->ekey); free(T->tkey);
    free(T->near_ptr); free(T->near_idx); free(T->inter_ptr); free(T->inter_idx);
    free(T);
}

/* ------------------------------------------------------------------ */
/* Multi-indices gamma = (a,b,c), |gamma| <= n, in graded order:       */
/* degree, then a descending, then b descending.                       */
/* ------------------------------------------------------------------ */
#define MAXD 32

static int ncoef(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }

static int midx(int a, int b, int c)
{
    int n = a + b + c;
    return n * (n + 1) * (n + 2) / 6 + (n - a) * (n - a + 1) / 2 + (n - a - b);
}

static void mexps(int p, int (*e)[3])
{
    for (int n = 0; n <= p; n++)
        for (int a = n; a >= 0; a--)
            for (int b = n - a; b >= 0; b--) {
                int i = midx(a, b, n - a - b);
                e[i][0] = a; e[i][1] = b; e[i][2] = n - a - b;
            }
}

/* ------------------------------------------------------------------ */
/* Section 3.3: derivatives D_gamma = d^gamma G(r) for |gamma| <= H.   */
/* Radial sequence G^(h) = (R^-1 d/dR)^h G: Laplace G^(h+1) =          */
/* -(2h+1) G^(h)/R^2; Helmholtz G^(h+1) = -((2h+1) G^(h) + k^2         */
/* G^(h-1))/R^2 for h >= 1 (index h-1 read for the printed q-1), with  */
/* G^(1) = (jkR - 1) e^{jkR}/(4 pi R^3).  Cartesian derivatives by Eq. */
/* 12 (the y-rows' "y^m" read as "y^n"), h descending (three steps).   */
/* ------------------------------------------------------------------ */
static void derivs(int green, double k, const double r[3], int H, cplx *D /* ncoef(H) */)
{
    int nc = ncoef(H);
    if (green == OR_R2) {
        for (int i = 0; i < nc; i++) D[i] = 0.0;
        D[0] = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        if (H >= 1) { D[midx(1, 0, 0)] = 2 * r[0]; D[midx(0, 1, 0)] = 2 * r[1]; D[midx(0, 0, 1)] = 2 * r[2]; }
        if (H >= 2) { D[midx(2, 0, 0)] = 2; D[midx(0, 2, 0)] = 2; D[midx(0, 0, 2)] = 2; }
        return;
    }
    static __thread int (*ex)[3] = NULL;
    static __thread int exH = -1;
    if (exH < H) {
        free(ex);
        ex = malloc(ncoef(H) * sizeof *ex);
        mexps(H, ex);
        exH = H;
    }
    double R2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2], R = sqrt(R2);
    cplx g[MAXD + 2];
    if (green == OR_LAPLACE) {
        g[0] = 1.0 / (4.0 * PI * R);
        for (int h = 0; h < H; h++) g[h + 1] = -(2.0 * h + 1.0) * g[h] / R2;
    } else {
        cplx e = cexp(I * k * R);
        g[0] = e / (4.0 * PI * R);
        if (H >= 1) g[1] = (I * k * R - 1.0) * e / (4.0 * PI * R * R2);
        for (int h = 1; h < H; h++) g[h + 1] = -((2.0 * h + 1.0) * g[h] + k * k * g[h - 1]) / R2;
    }
    cplx *prev = malloc(nc * sizeof(cplx)), *cur = malloc(nc * sizeof(cplx));
    /* step 1 and 2: level h holds d^gamma G^(h) for |gamma| <= H - h */
    prev[0] = g[H];
    for (int h = H - 1; h >= 0; h--) {
        int m = ncoef(H - h);
        cur[0] = g[h];
        for (int i = 1; i < m; i++) {
            int a = ex[i][0], b = ex[i][1], c = ex[i][2];
            int d = a > 0 ? 0 : (b > 0 ? 1 : 2);
            int al[3] = {a, b, c};
            al[d]--; /* gamma = alpha + e_d */
            cplx v = r[d] * prev[midx(al[0], al[1], al[2])];
            if (al[d] > 0) {
                int am[3] = {al[0], al[1], al[2]};
                am[d]--;
                v += (double)al[d] * prev[midx(am[0], am[1], am[2])];
            }
            cur[i] = v;
        }
        cplx *t = prev; prev = cur; cur = t;
    }
    /* step 3 */
    memcpy(D, prev, nc * sizeof(cplx));
    free(prev); free(cur);
}

void or_derivs(int green, double k, const double *r, int H, double *D)
{
    derivs(green, k, r, H, (cplx *)D);
}

/* ------------------------------------------------------------------ */
/* Section 3.2 and 3.6: the fast matrix product.                       */
/*  - moments I_alpha about a box centre (Eqs. 6-8), from the 7-point  */
/*    rule's points; for the double layer the moment of n1.grad_y of   */
/*    the monomial (a reading: the paper writes the single layer only) */
/*  - coefficient shift (Eq. 10), expansion shift with the binomial    */
/*    factors (Eq. 11 read with them), local expansion (Eq. 9 read as  */
/*    F_b = sum_a (-1)^|a| d^(a+b)G M_a / (a! b!))                    */
/*  - near field by direct 7-point sums over the near-list boxes, plus */
/*    the accurate-minus-regular correction on singular and near-      */
/*    singular pairs.                                                  */
/* ------------------------------------------------------------------ */
static double fact(int n) { double f = 1.0; for (int i = 2; i <= n; i++) f *= i; return f; }

static double binom(int n, int k) { return fact(n) / (fact(k) * fact(n - k)); }

static double ipow(double x, int n) { double r = 1.0; for (int i = 0; i < n; i++) r *= x; return r; }

/* Section 3.6: the expansion order may depend on the level, L_l =          */
/* min(L_max, L_min + l_max - l) with l_max the deepest level of the tree;  */
/* order_min <= 0 keeps L_max everywhere.  Every expansion of a box at      */
/* level l has order L_l: moments and locals past it are never formed, so   */
/* a parent's moments come from its children's truncated moments (Eq. 10)   */
/* and a child's locals are the parent's truncated to the child's order     */
/* (Eq. 11); a translation (Eq. 9) maps order L_source to order L_target.   */
int or_fmm_matvec(const void *h, const double *xyz, const int32_t *elem, const int32_t *elem_dofs,
                  const int32_t *dof_node, int64_t n_el, int64_t n_dof, int nn, int green, double k,
                  int order, int order_min, int op, const double *x_in, double *y_out)
{
    const otree_t *T = h;
    const cplx *x = (const cplx *)x_in;
    cplx *y = (cplx *)y_out;
    mesh_t m = {xyz, elem, elem_dofs, dof_node, n_el, n_dof, nn};
    int p = order, P = ncoef(p), P2 = ncoef(2 * p);
    int dbl = (op == OP_K || op == OP_A || op == OP_K_REG);
    int regular_only = (op == OP_S_REG || op == OP_K_REG);
    int (*ex)[3] = malloc(P2 * sizeof *ex);
    mexps(2 * p, ex);

    /* Source points of the 7-point rule and their strengths, in the tree's  */
    /* source order: the points of sorted source s are so[s] .. so[s+1]-1.    */
    /* Sources are the elements (7 points each, strength wJ sum_a L_a x_a),   */
    /* or in the literal tree the DOFs: DOF i's basis function over its       */
    /* element patch, 7 points of every element e holding it in slot a, with  */
    /* strength wJ L_a x_i.                                                    */
    rule_t reg;
    rule_regular(&reg);
    int64_t ns = T->n_el; /* sorted sources */
    int64_t *so = malloc((ns + 1) * sizeof *so);
    int64_t *ip = NULL, *iv = NULL; /* DOF -> incidences nn*e + a (literal tree) */
    if (T->literal) {
        ip = calloc(n_dof + 1, sizeof *ip);
        for (int64_t i = 0; i < nn * n_el; i++) ip[elem_dofs[i] + 1]++;
        for (int64_t i = 0; i < n_dof; i++) ip[i + 1] += ip[i];
        int64_t *fill = malloc((n_dof + 1) * sizeof *fill);
        memcpy(fill, ip, (n_dof + 1) * sizeof *fill);
        iv = malloc((nn * n_el + 1) * sizeof *iv);
        for (int64_t i = 0; i < nn * n_el; i++) iv[fill[elem_dofs[i]]++] = i;
        free(fill);
    }
    so[0] = 0;
    for (int64_t s = 0; s < ns; s++)
        so[s + 1] = so[s] + (T->literal ? 7 * (ip[T->eperm[s] + 1] - ip[T->eperm[s]]) : 7);
    int64_t nq = so[ns];
    double (*qy)[3] = malloc((nq + 1) * sizeof *qy), (*qn)[3] = malloc((nq + 1) * sizeof *qn);
    cplx *qs = malloc((nq + 1) * sizeof(cplx));
    for (int64_t s = 0; s < ns; s++) {
        int64_t o = so[s];
        if (!T->literal) {
            int64_t e = T->eperm[s];
            double X[6][3];
            load_elem(nn, xyz, elem + nn * e, X);
            for (int q = 0; q < 7; q++) {
                double L[6], J;
                elem_point(nn, X, reg.s[q], reg.t[q], qy[o + q], qn[o + q], &J, L);
                cplx sig = 0.0;
                for (int a = 0; a < nn; a++) sig += L[a] * x[elem_dofs[nn * e + a]];
                qs[o + q] = sig * (reg.w[q] * J);
            }
            continue;
        }
        int64_t i = T->eperm[s];
        for (int64_t p = ip[i]; p < ip[i + 1]; p++, o += 7) {
            int64_t e = iv[p] / nn;
            int a = (int)(iv[p] % nn);
            double X[6][3];
            load_elem(nn, xyz, elem + nn * e, X);
            for (int q = 0; q < 7; q++) {
                double L[6], J;
                elem_point(nn, X, reg.s[q], reg.t[q], qy[o + q], qn[o + q], &J, L);
                qs[o + q] = x[i] * (L[a] * (reg.w[q] * J));
            }
        }
    }
    cplx *M = calloc(T->n_box * P, sizeof(cplx)), *F = calloc(T->n_box * P, sizeof(cplx));
    /* number of coefficients of each box's expansions */
    int lmax = 0;
    for (int64_t b = 0; b < T->n_box; b++)
        if (T->box[b].level > lmax) lmax = T->box[b].level;
    int *nc = malloc(T->n_box * sizeof *nc);
    for (int64_t b = 0; b < T->n_box; b++) {
        int Lb = p;
        if (order_min > 0 && order_min + lmax - T->box[b].level < p) Lb = order_min + lmax - T->box[b].level;
        nc[b] = ncoef(Lb);
    }
    /* P2M at leaves */
    for (int64_t b = 0; b < T->n_box; b++) {
        const obox_t *B_ = &T->box[b];
        if (!B_->leaf) continue;
        for (int64_t q = so[B_->eb]; q < so[B_->ee]; q++) {
            double d[3] = {qy[q][0] - B_->c[0], qy[q][1] - B_->c[1], qy[q][2] - B_->c[2]};
            for (int i = 0; i < nc[b]; i++) {
                int a = ex[i][0], bb = ex[i][1], c = ex[i][2];
                if (!dbl) {
                    M[b * P + i] += qs[q] * ipow(d[0], a) * ipow(d[1], bb) * ipow(d[2], c);
                } else {
                    double v = 0.0;
                    if (a) v += qn[q][0] * a * ipow(d[0], a - 1) * ipow(d[1], bb) * ipow(d[2], c);
                    if (bb) v += qn[q][1] * bb * ipow(d[0], a) * ipow(d[1], bb - 1) * ipow(d[2], c);
                    if (c) v += qn[q][2] * c * ipow(d[0], a) * ipow(d[1], bb) * ipow(d[2], c - 1);
                    M[b * P + i] += qs[q] * v;
                }
            }
        }
    }
    /* M2M, Eq. 10, bottom-up */
    for (int64_t b = T->n_box - 1; b >= 1; b--) {
        const obox_t *C = &T->box[b];
        int64_t pb = C->parent;
        const obox_t *Pa = &T->box[pb];
        double d[3] = {C->c[0] - Pa->c[0], C->c[1] - Pa->c[1], C->c[2] - Pa->c[2]};
        for (int i = 0; i < nc[pb]; i++) {
            int a = ex[i][0], bb = ex[i][1], c = ex[i][2];
            cplx acc = 0.0;
            for (int q = 0; q <= a; q++)
                for (int r = 0; r <= bb; r++)
                    for (int s = 0; s <= c; s++)
                        acc += binom(a, q) * binom(bb, r) * binom(c, s) * ipow(d[0], q) * ipow(d[1], r) *
                               ipow(d[2], s) * M[b * P + midx(a - q, bb - r, c - s)];
            M[pb * P + i] += acc;
        }
    }
    /* M2L, Eq. 9, and L2L, Eq. 11, top-down */
    double *fa = malloc(P * sizeof(double));
    for (int i = 0; i < P; i++) fa[i] = fact(ex[i][0]) * fact(ex[i][1]) * fact(ex[i][2]);
    for (int64_t b = 0; b < T->n_box; b++) {
        const obox_t *B_ = &T->box[b];
        if (b > 0) {
            const obox_t *Pa = &T->box[B_->parent];
            double d[3] = {B_->c[0] - Pa->c[0], B_->c[1] - Pa->c[1], B_->c[2] - Pa->c[2]};
            for (int i = 0; i < nc[b]; i++) {
                int a = ex[i][0], bb = ex[i][1], c = ex[i][2];
                cplx acc = 0.0;
                for (int j = 0; j < nc[B_->parent]; j++) {
                    int a2 = ex[j][0], b2 = ex[j][1], c2 = ex[j][2];
                    if (a2 < a || b2 < bb || c2 < c) continue;
                    acc += binom(a2, a) * binom(b2, bb) * binom(c2, c) * ipow(d[0], a2 - a) *
                           ipow(d[1], b2 - bb) * ipow(d[2], c2 - c) * F[B_->parent * P + j];
                }
                F[b * P + i] += acc;
            }
        }
        cplx *D = malloc(P2 * sizeof(cplx));
        for (int64_t j = T->inter_ptr[b]; j < T->inter_ptr[b + 1]; j++) {
            const obox_t *S_ = &T->box[T->inter_idx[j]];
            double r[3] = {B_->c[0] - S_->c[0], B_->c[1] - S_->c[1], B_->c[2] - S_->c[2]};
            derivs(green, k, r, 2 * p, D);
            for (int i = 0; i < nc[b]; i++) {
                cplx acc = 0.0;
                for (int a = 0; a < nc[T->inter_idx[j]]; a++) {
                    int g0 = ex[i][0] + ex[a][0], g1 = ex[i][1] + ex[a][1], g2 = ex[i][2] + ex[a][2];
                    double sg = ((ex[a][0] + ex[a][1] + ex[a][2]) & 1) ? -1.0 : 1.0;
                    acc += sg * D[midx(g0, g1, g2)] * M[T->inter_idx[j] * P + a] / fa[a];
                }
                F[b * P + i] += acc / fa[i];
            }
        }
        free(D);
    }
    /* L2P + near field + corrections, per target */
    cplx *yo = calloc(n_dof, sizeof(cplx));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < T->n_box; b++) {
        const obox_t *B_ = &T->box[b];
        if (!B_->leaf) continue;
        for (int64_t t = B_->tb; t < B_->te; t++) {
            int64_t i = T->tperm[t];
            const double *xi = xyz + 3 * (int64_t)dof_node[i];
            double d[3] = {xi[0] - B_->c[0], xi[1] - B_->c[1], xi[2] - B_->c[2]};
            cplx acc = 0.0;
            for (int j = 0; j < nc[b]; j++)
                acc += F[b * P + j] * ipow(d[0], ex[j][0]) * ipow(d[1], ex[j][1]) * ipow(d[2], ex[j][2]);
            for (int64_t j = T->near_ptr[b]; j < T->near_ptr[b + 1]; j++) {
                const obox_t *S_ = &T->box[T->near_idx[j]];
                for (int64_t q = so[S_->eb]; q < so[S_->ee]; q++) {
                    cplx G, dG;
                    kernel(green, k, xi, qy[q], qn[q], &G, &dG);
                    acc += (dbl ? dG : G) * qs[q];
                }
            }
            yo[i] = acc;
        }
    }
    /* accurate-minus-regular corrections on every singular / near-singular pair */
    if (!regular_only && green != OR_R2) {
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t i = 0; i < n_dof; i++) {
            const double *xi = xyz + 3 * (int64_t)dof_node[i];
            cplx acc = 0.0;
            for (int64_t e = 0; e < n_el; e++) {
                int param;
                if (classify(nn, xyz, elem + nn * e, dof_node[i], xi, &param) == CL_REGULAR) continue;
                cplx S[6], K[6], Sr[6], Kr[6];
                pair_integrals(nn, xyz, elem + nn * e, dof_node[i], xi, green, k, S, K, Sr, Kr);
                for (int a = 0; a < nn; a++)
                    acc += (dbl ? (K[a] - Kr[a]) : (S[a] - Sr[a])) * x[elem_dofs[nn * e + a]];
            }
            yo[i] += acc;
        }
    }
    /* combine */
    double *c = NULL;
    if (op == OP_A) {
        c = malloc(n_dof * sizeof(double));
        int64_t *rows = malloc(n_dof * sizeof(int64_t));
        for (int64_t i = 0; i < n_dof; i++) rows[i] = i;
        or_free_term(xyz, elem, elem_dofs, dof_node, n_el, n_dof, nn, rows, n_dof, c);
        free(rows);
    }
    for (int64_t i = 0; i < n_dof; i++) {
        if (op == OP_A) y[i] = c[i] * x[i] - yo[i];
        else if (op == OP_RHS) y[i] = -yo[i];
        else y[i] = yo[i];
    }
    (void)m;
    free(c); free(yo); free(fa); free(M); free(F); free(nc); free(qy); free(qn); free(qs); free(ex);
    free(so); free(ip); free(iv);
    return 0;
}

/* Section 3.2 pieces exported for the shift-identity pins. */
void or_mono_moments(int p, const double *c, const double *pts, const double *w, int64_t n, double *M)
{
    int P = ncoef(p);
    int (*ex)[3] = malloc(P * sizeof *ex);
    mexps(p, ex);
    for (int i = 0; i < P; i++) {
        double acc = 0.0;
        for (int64_t q = 0; q < n; q++)
            acc += w[q] * ipow(pts[3 * q] - c[0], ex[i][0]) * ipow(pts[3 * q + 1] - c[1], ex[i][1]) *
                   ipow(pts[3 * q + 2] - c[2], ex[i][2]);
        M[i] = acc;
    }
    free(ex);
}

void or_m2m(int p, const double *d /* child - parent */, const double *Mc, double *Mp)
{
    int P = ncoef(p);
    int (*ex)[3] = malloc(P * sizeof *ex);
    mexps(p, ex);
    for (int i = 0; i < P; i++) {
        int a = ex[i][0], b = ex[i][1], c = ex[i][2];
        double acc = 0.0;
        for (int q = 0; q <= a; q++)
            for (int r = 0; r <= b; r++)
                for (int s = 0; s <= c; s++)
                    acc += binom(a, q) * binom(b, r) * binom(c, s) * ipow(d[0], q) * ipow(d[1], r) *
                           ipow(d[2], s) * Mc[midx(a - q, b - r, c - s)];
        Mp[i] = acc;
    }
    free(ex);
}

void or_l2l(int p, const double *d /* child - parent */, const double *Fp, double *Fc)
{
    int P = ncoef(p);
    int (*ex)[3] = malloc(P * sizeof *ex);
    mexps(p, ex);
    for (int i = 0; i < P; i++) {
        double acc = 0.0;
        for (int j = 0; j < P; j++) {
            if (ex[j][0] < ex[i][0] || ex[j][1] < ex[i][1] || ex[j][2] < ex[i][2]) continue;
            acc += binom(ex[j][0], ex[i][0]) * binom(ex[j][1], ex[i][1]) * binom(ex[j][2], ex[i][2]) *
                   ipow(d[0], ex[j][0] - ex[i][0]) * ipow(d[1], ex[j][1] - ex[i][1]) *
                   ipow(d[2], ex[j][2] - ex[i][2]) * Fp[j];
        }
        Fc[i] = acc;
    }
    free(ex);
}

void or_multi_index(int p, int32_t *e)
{
    int P = ncoef(p);
    int (*ex)[3] = malloc(P * sizeof *ex);
    mexps(p, ex);
    for (int i = 0; i < P; i++) { e[3 * i] = ex[i][0]; e[3 * i + 1] = ex[i][1]; e[3 * i + 2] = ex[i][2]; }
    free(ex);
}
