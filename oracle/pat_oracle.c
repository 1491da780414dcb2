/*
 * Plain CPU FP64 oracle for the matrix-free RTO sampler of
 * "3D Uncertainty Quantification for Photoacoustic Tomography" (arXiv 2607.21373).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct reference
 * that the GPU library is checked against.  Only the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load it; the product never does.
 * It shares no code with the GPU library.
 *
 * Everything is float64, built with -ffp-contract=off.  Multi-vectors with R
 * right-hand sides are stored node-major, RHS fastest: x[i*R + r].  Parallel
 * loops run over independent rows only, and every reduction is a sequential sum
 * in index order, so results are bitwise identical for any thread count.
 *
 * What each part follows in the paper:
 *   assembly            Sec. 3, eq. (semi-discrete) and the matrix definitions
 *                       below it; lumped mass M_L = diag(M 1) (Sec. 3)
 *   sensor operator Pi  Sec. 3, eq. (lagrange): P1 interpolation at the sensor
 *                       point (injection when the sensor is a node)
 *   forward step        Sec. 3, eq. (fully-discrete) with M replaced by M_L
 *   forward map G       Sec. 3, eq. (discrete-wave-matrix): y^n = Pi z^n, n=1..N_T
 *   transpose step      Sec. 5.1, eq. (adjoint-verlet); App. B
 *   transpose map G^T   Sec. 5.1, eqs. (transpose-definition), (backward-recursion)
 *   G_ext, b            Sec. 5, eq. (extended-matrices); residual and transpose
 *                       action eqs. (lsqr-residual), (lsqr-transpose-action)
 *   CGLS                least-squares solve of eq. (normal-equations), with full
 *                       reorthogonalisation of the normal-equation residuals
 *   LSQR                the same least squares by Paige and Saunders' Golub-Kahan
 *                       bidiagonalisation, the solver named in Sec. 5 and Algorithm 1
 *   RTO sample          Sec. 5, eq. (optimization); Algorithm 1
 *   mean / std          Sec. 6.2, eq. (ergodic)
 *   perturbations       the standard-normal draws eta, xi of Algorithm 1 when the
 *                       sampler makes its own: Philox4x64-10 (Salmon, Moraes, Dror
 *                       and Shaw, SC'11) followed by the Box-Muller transform
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int n;            /* number of rows (= columns) */
    int64_t nnz;
    int64_t *rowptr;  /* [n+1] */
    int *col;         /* [nnz], ascending within a row */
    double *val;      /* [nnz] */
} ocsr;

typedef struct {
    int n_nodes, n_obs, n_steps;
    double dt;
    ocsr K;    /* [K]_mn = c^2 int grad phi_m . grad phi_n */
    ocsr K1;   /* same with c = 1 (used by the prior) */
    ocsr B;    /* [B]_mn = (1/c) int_{boundary} phi_m phi_n ; all zero when reflecting */
    double *mL;     /* lumped mass, diag(M 1) */
    int *snode;     /* [n_obs][4] */
    double *sw;     /* [n_obs][4] interpolation weights */
} oproblem;

/* ------------------------------------------------------------------ */
/* Sparse pattern construction                                         */
/* ------------------------------------------------------------------ */

static int cmp_int(const void *a, const void *b) {
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

/* Build a CSR pattern from groups of `k` node ids (every pair in a group couples). */
static int pattern_from_groups(int n, int64_t ngroups, int k, const int *groups, ocsr *A) {
    int64_t *cnt = calloc((size_t)n + 1, sizeof(int64_t));
    if (!cnt) return -1;
    for (int64_t g = 0; g < ngroups; ++g)
        for (int a = 0; a < k; ++a) cnt[groups[g * k + a] + 1] += k;
    for (int i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    int *tmp = malloc(sizeof(int) * (size_t)(cnt[n] > 0 ? cnt[n] : 1));
    int64_t *fill = malloc(sizeof(int64_t) * (size_t)n);
    if (!tmp || !fill) { free(cnt); free(tmp); free(fill); return -1; }
    for (int i = 0; i < n; ++i) fill[i] = cnt[i];
    for (int64_t g = 0; g < ngroups; ++g)
        for (int a = 0; a < k; ++a) {
            int row = groups[g * k + a];
            for (int b = 0; b < k; ++b) tmp[fill[row]++] = groups[g * k + b];
        }
    A->n = n;
    A->rowptr = malloc(sizeof(int64_t) * ((size_t)n + 1));
    A->rowptr[0] = 0;
    /* sort and deduplicate each row */
    int64_t total = 0;
    for (int i = 0; i < n; ++i) {
        int64_t s = cnt[i], e = cnt[i + 1];
        qsort(tmp + s, (size_t)(e - s), sizeof(int), cmp_int);
        int64_t u = 0;
        for (int64_t t = s; t < e; ++t)
            if (u == 0 || tmp[s + u - 1] != tmp[t]) tmp[s + u++] = tmp[t];
        fill[i] = u;
        total += u;
        A->rowptr[i + 1] = total;
    }
    A->nnz = total;
    A->col = malloc(sizeof(int) * (size_t)(total > 0 ? total : 1));
    A->val = calloc((size_t)(total > 0 ? total : 1), sizeof(double));
    for (int i = 0; i < n; ++i)
        memcpy(A->col + A->rowptr[i], tmp + cnt[i], sizeof(int) * (size_t)fill[i]);
    free(tmp); free(fill); free(cnt);
    return 0;
}

/* Location of column j in row i (binary search); -1 if absent. */
static int64_t csr_find(const ocsr *A, int i, int j) {
    int64_t lo = A->rowptr[i], hi = A->rowptr[i + 1] - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (A->col[mid] == j) return mid;
        if (A->col[mid] < j) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

static void csr_free(ocsr *A) { free(A->rowptr); free(A->col); free(A->val); memset(A, 0, sizeof(*A)); }

/* ------------------------------------------------------------------ */
/* Geometry                                                            */
/* ------------------------------------------------------------------ */

static void sub3(const double *a, const double *b, double *o) { o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2]; }
static void cross3(const double *a, const double *b, double *o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Gradients of the four barycentric (P1 nodal basis) functions of a tetrahedron
 * and its signed 6*volume.  grad lambda_1 = (e2 x e3)/det, etc., with
 * e_k = x_k - x_0 and det = e1 . (e2 x e3); grad lambda_0 = -sum of the others. */
static double tet_gradients(const double *X, const int *t, double g[4][3]) {
    double e1[3], e2[3], e3[3], c23[3], c31[3], c12[3];
    sub3(X + 3 * t[1], X + 3 * t[0], e1);
    sub3(X + 3 * t[2], X + 3 * t[0], e2);
    sub3(X + 3 * t[3], X + 3 * t[0], e3);
    cross3(e2, e3, c23); cross3(e3, e1, c31); cross3(e1, e2, c12);
    double det = dot3(e1, c23);
    for (int d = 0; d < 3; ++d) {
        g[1][d] = c23[d] / det;
        g[2][d] = c31[d] / det;
        g[3][d] = c12[d] / det;
        g[0][d] = -(g[1][d] + g[2][d] + g[3][d]);
    }
    return det;
}

/* ------------------------------------------------------------------ */
/* Boundary faces: faces owned by exactly one tetrahedron              */
/* ------------------------------------------------------------------ */

typedef struct { int a, b, c, tet; } oface;

static int cmp_face(const void *x, const void *y) {
    const oface *f = x, *g = y;
    if (f->a != g->a) return (f->a > g->a) - (f->a < g->a);
    if (f->b != g->b) return (f->b > g->b) - (f->b < g->b);
    if (f->c != g->c) return (f->c > g->c) - (f->c < g->c);
    return (f->tet > g->tet) - (f->tet < g->tet);
}

static void sort3(int *v) {
    int t;
    if (v[0] > v[1]) { t = v[0]; v[0] = v[1]; v[1] = t; }
    if (v[1] > v[2]) { t = v[1]; v[1] = v[2]; v[2] = t; }
    if (v[0] > v[1]) { t = v[0]; v[0] = v[1]; v[1] = t; }
}

/* Returns the number of boundary faces; fills faces[nb] (sorted node triples + owner). */
static int64_t boundary_faces(int64_t E, const int *tets, oface **out) {
    static const int fl[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
    oface *all = malloc(sizeof(oface) * (size_t)(4 * E));
    for (int64_t e = 0; e < E; ++e)
        for (int f = 0; f < 4; ++f) {
            int v[3] = {tets[4 * e + fl[f][0]], tets[4 * e + fl[f][1]], tets[4 * e + fl[f][2]]};
            sort3(v);
            all[4 * e + f] = (oface){v[0], v[1], v[2], (int)e};
        }
    qsort(all, (size_t)(4 * E), sizeof(oface), cmp_face);
    int64_t nb = 0;
    for (int64_t i = 0; i < 4 * E;) {
        int64_t j = i + 1;
        while (j < 4 * E && all[j].a == all[i].a && all[j].b == all[i].b && all[j].c == all[i].c) ++j;
        if (j - i == 1) all[nb++] = all[i];
        i = j;
    }
    *out = all;
    return nb;
}

/* ------------------------------------------------------------------ */
/* Problem construction                                                */
/* ------------------------------------------------------------------ */

/* Point location: the tetrahedron whose smallest barycentric coordinate of x is
 * largest (first such tetrahedron on ties).  Returns that smallest coordinate. */
static double locate(int64_t E, const int *tets, const double *X, const double *x, int *best_tet, double lam_out[4]) {
    double best = -1e300;
    *best_tet = -1;
    for (int64_t e = 0; e < E; ++e) {
        const int *t = tets + 4 * e;
        double e1[3], e2[3], e3[3], d[3], c[3], lam[4];
        sub3(X + 3 * t[1], X + 3 * t[0], e1);
        sub3(X + 3 * t[2], X + 3 * t[0], e2);
        sub3(X + 3 * t[3], X + 3 * t[0], e3);
        sub3(x, X + 3 * t[0], d);
        cross3(e2, e3, c);
        double det = dot3(e1, c);
        lam[1] = dot3(d, c) / det;
        cross3(e3, e1, c);
        lam[2] = dot3(d, c) / det;
        cross3(e1, e2, c);
        lam[3] = dot3(d, c) / det;
        lam[0] = 1.0 - lam[1] - lam[2] - lam[3];
        double m = lam[0];
        for (int k = 1; k < 4; ++k) if (lam[k] < m) m = lam[k];
        if (m > best) {
            best = m;
            *best_tet = (int)e;
            for (int k = 0; k < 4; ++k) lam_out[k] = lam[k];
        }
    }
    return best;
}

/* Create the discrete problem.
 *   coords[N][3], tets[E][4]: P1 mesh.  c_tet[E] wave speed per element or NULL (c = 1).
 *   absorbing: 1 = first-order absorbing boundary (B assembled), 0 = reflecting (B = 0).
 *   Sensors: either sensor_nodes[n_obs] (node ids) or sensor_pos[n_obs][3] (points).
 * Returns NULL on failure (a sensor outside the mesh, bad input). */
oproblem *orc_create(int N, const double *coords, int64_t E, const int *tets, const double *c_tet,
                     int absorbing, int n_obs, const int *sensor_nodes, const double *sensor_pos,
                     double dt, int n_steps) {
    oproblem *P = calloc(1, sizeof(oproblem));
    P->n_nodes = N; P->n_obs = n_obs; P->n_steps = n_steps; P->dt = dt;
    for (int64_t e = 0; e < 4 * E; ++e)
        if (tets[e] < 0 || tets[e] >= N) { free(P); return NULL; }

    /* stiffness matrices K (c^2) and K1 (c = 1), lumped mass */
    pattern_from_groups(N, E, 4, tets, &P->K);
    pattern_from_groups(N, E, 4, tets, &P->K1);
    P->mL = calloc((size_t)N, sizeof(double));
    for (int64_t e = 0; e < E; ++e) {
        const int *t = tets + 4 * e;
        double g[4][3];
        double det = tet_gradients(coords, t, g);
        double vol = fabs(det) / 6.0;
        double c = c_tet ? c_tet[e] : 1.0;
        for (int a = 0; a < 4; ++a) {
            P->mL[t[a]] += vol / 4.0;
            for (int b = 0; b < 4; ++b) {
                double kab = vol * dot3(g[a], g[b]);
                int64_t pos = csr_find(&P->K, t[a], t[b]);
                P->K.val[pos] += c * c * kab;
                P->K1.val[pos] += kab;
            }
        }
    }

    /* boundary mass: consistent P1 face mass (area/12)(1 + delta_ab), scaled by 1/c
     * of the tetrahedron that owns the face */
    oface *faces = NULL;
    int64_t nb = absorbing ? boundary_faces(E, tets, &faces) : 0;
    int *fnodes = malloc(sizeof(int) * (size_t)(3 * (nb > 0 ? nb : 1)));
    for (int64_t f = 0; f < nb; ++f) {
        fnodes[3 * f] = faces[f].a; fnodes[3 * f + 1] = faces[f].b; fnodes[3 * f + 2] = faces[f].c;
    }
    pattern_from_groups(N, nb, 3, fnodes, &P->B);
    for (int64_t f = 0; f < nb; ++f) {
        const int *v = fnodes + 3 * f;
        double e1[3], e2[3], cr[3];
        sub3(coords + 3 * v[1], coords + 3 * v[0], e1);
        sub3(coords + 3 * v[2], coords + 3 * v[0], e2);
        cross3(e1, e2, cr);
        double area = 0.5 * sqrt(dot3(cr, cr));
        double c = c_tet ? c_tet[faces[f].tet] : 1.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                P->B.val[csr_find(&P->B, v[a], v[b])] += (a == b ? 2.0 : 1.0) * area / 12.0 / c;
    }
    free(fnodes); free(faces);

    /* sensor interpolation rows */
    P->snode = malloc(sizeof(int) * 4 * (size_t)(n_obs > 0 ? n_obs : 1));
    P->sw = malloc(sizeof(double) * 4 * (size_t)(n_obs > 0 ? n_obs : 1));
    int bad = 0;
    if (sensor_nodes) {
        for (int s = 0; s < n_obs; ++s) {
            if (sensor_nodes[s] < 0 || sensor_nodes[s] >= N) bad = 1;
            for (int k = 0; k < 4; ++k) { P->snode[4 * s + k] = sensor_nodes[s]; P->sw[4 * s + k] = k == 0 ? 1.0 : 0.0; }
        }
    } else {
#pragma omp parallel for schedule(dynamic, 1)
        for (int s = 0; s < n_obs; ++s) {
            int te; double lam[4];
            double m = locate(E, tets, coords, sensor_pos + 3 * s, &te, lam);
            if (te < 0 || m < -1e-10) {
#pragma omp atomic write
                bad = 1;
                continue;
            }
            for (int k = 0; k < 4; ++k) { P->snode[4 * s + k] = tets[4 * te + k]; P->sw[4 * s + k] = lam[k]; }
        }
    }
    if (bad) {
        csr_free(&P->K); csr_free(&P->K1); csr_free(&P->B);
        free(P->mL); free(P->snode); free(P->sw); free(P);
        return NULL;
    }
    return P;
}

void orc_destroy(oproblem *P) {
    if (!P) return;
    csr_free(&P->K); csr_free(&P->K1); csr_free(&P->B);
    free(P->mL); free(P->snode); free(P->sw); free(P);
}

/* Export sizes and arrays (for tests). which: 0 = K, 1 = K1, 2 = B. */
int64_t orc_nnz(const oproblem *P, int which) { return which == 0 ? P->K.nnz : which == 1 ? P->K1.nnz : P->B.nnz; }
void orc_get_csr(const oproblem *P, int which, int64_t *rowptr, int *col, double *val) {
    const ocsr *A = which == 0 ? &P->K : which == 1 ? &P->K1 : &P->B;
    memcpy(rowptr, A->rowptr, sizeof(int64_t) * ((size_t)A->n + 1));
    memcpy(col, A->col, sizeof(int) * (size_t)A->nnz);
    memcpy(val, A->val, sizeof(double) * (size_t)A->nnz);
}
void orc_get_mass(const oproblem *P, double *mL) { memcpy(mL, P->mL, sizeof(double) * (size_t)P->n_nodes); }
void orc_get_sensors(const oproblem *P, int *snode, double *sw) {
    memcpy(snode, P->snode, sizeof(int) * 4 * (size_t)P->n_obs);
    memcpy(sw, P->sw, sizeof(double) * 4 * (size_t)P->n_obs);
}

/* ------------------------------------------------------------------ */
/* Sparse products, row by row                                         */
/* ------------------------------------------------------------------ */

/* acc[r] = sum_k A_ik x[col_k][r] for one row i */
static inline void row_product(const ocsr *A, int i, int R, const double *restrict x, double *restrict acc) {
    for (int r = 0; r < R; ++r) acc[r] = 0.0;
    for (int64_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k) {
        const double a = A->val[k];
        const double *xj = x + (size_t)A->col[k] * R;
        for (int r = 0; r < R; ++r) acc[r] += a * xj[r];
    }
}

/* y = A x for multi-vectors */
void orc_spmv(const ocsr *A, int R, const double *x, double *y) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < A->n; ++i) row_product(A, i, R, x, y + (size_t)i * R);
}

/* ------------------------------------------------------------------ */
/* Forward Stormer-Verlet step, eq. (fully-discrete) with M -> M_L     */
/* ------------------------------------------------------------------ */

/* One step z^n = (p, v) -> z^{n+1}; p, v updated in place.
 * work: 2*N*R doubles (p^{n+1/2} and the new v). */
void orc_step(const oproblem *P, int R, double *p, double *v, double *work) {
    const int N = P->n_nodes;
    const double dt = P->dt;
    double *ph = work, *vn = work + (size_t)N * R;
    /* p^{n+1/2} = p^n + (dt/2) v^n */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < N; ++i)
        for (int r = 0; r < R; ++r) ph[(size_t)i * R + r] = p[(size_t)i * R + r] + 0.5 * dt * v[(size_t)i * R + r];
    /* M_L v^{n+1} = M_L v^n - dt K p^{n+1/2} - dt B v^n */
#pragma omp parallel
    {
        double *kp = malloc(sizeof(double) * (size_t)R), *bv = malloc(sizeof(double) * (size_t)R);
#pragma omp for schedule(static)
        for (int i = 0; i < N; ++i) {
            row_product(&P->K, i, R, ph, kp);
            row_product(&P->B, i, R, v, bv);
            for (int r = 0; r < R; ++r) {
                double rhs = P->mL[i] * v[(size_t)i * R + r] - dt * kp[r] - dt * bv[r];
                vn[(size_t)i * R + r] = rhs / P->mL[i];
            }
        }
        free(kp); free(bv);
    }
    /* p^{n+1} = p^{n+1/2} + (dt/2) v^{n+1} */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < N; ++i)
        for (int r = 0; r < R; ++r) {
            v[(size_t)i * R + r] = vn[(size_t)i * R + r];
            p[(size_t)i * R + r] = ph[(size_t)i * R + r] + 0.5 * dt * vn[(size_t)i * R + r];
        }
}

/* y_s = sum_k w_sk p[node_sk] (Pi applied to the pressure part) */
static void observe(const oproblem *P, int R, const double *p, double *y) {
    for (int s = 0; s < P->n_obs; ++s)
        for (int r = 0; r < R; ++r) {
            double acc = 0.0;
            for (int k = 0; k < 4; ++k) acc += P->sw[4 * s + k] * p[(size_t)P->snode[4 * s + k] * R + r];
            y[(size_t)s * R + r] = acc;
        }
}

/* Forward map: y^n = Pi A^n z_0, z_0 = (p0, 0), n = 1..N_T.
 * p0 [N][R]; y [N_T][n_obs][R]. */
void orc_forward(const oproblem *P, int R, const double *p0, double *y) {
    const size_t NR = (size_t)P->n_nodes * R;
    double *p = malloc(sizeof(double) * NR), *v = calloc(NR, sizeof(double)), *w = malloc(sizeof(double) * 2 * NR);
    memcpy(p, p0, sizeof(double) * NR);
    for (int n = 1; n <= P->n_steps; ++n) {
        orc_step(P, R, p, v, w);
        observe(P, R, p, y + (size_t)(n - 1) * P->n_obs * R);
    }
    free(p); free(v); free(w);
}

/* ------------------------------------------------------------------ */
/* Transpose step, eq. (adjoint-verlet): A^T = S1^T S2^T S3^T S4^T      */
/* ------------------------------------------------------------------ */

/* (ph, vh) <- A_dt^T (ph, vh), in place.  work: N*R doubles (q). */
void orc_step_transpose(const oproblem *P, int R, double *ph, double *vh, double *work) {
    const int N = P->n_nodes;
    const double dt = P->dt;
    double *q = work;
    /* vh^{n+1/2} = vh^{n+1} + (dt/2) ph^{n+1};  M_L q = vh^{n+1/2} */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < N; ++i)
        for (int r = 0; r < R; ++r)
            q[(size_t)i * R + r] = (vh[(size_t)i * R + r] + 0.5 * dt * ph[(size_t)i * R + r]) / P->mL[i];
    /* ph^n = ph^{n+1/2} - dt K^T q ;  vh^n = (M_L - dt B^T) q + (dt/2) ph^n   (K, B symmetric) */
#pragma omp parallel
    {
        double *kq = malloc(sizeof(double) * (size_t)R), *bq = malloc(sizeof(double) * (size_t)R);
#pragma omp for schedule(static)
        for (int i = 0; i < N; ++i) {
            row_product(&P->K, i, R, q, kq);
            row_product(&P->B, i, R, q, bq);
            for (int r = 0; r < R; ++r) {
                double pn = ph[(size_t)i * R + r] - dt * kq[r];
                ph[(size_t)i * R + r] = pn;
                vh[(size_t)i * R + r] = (P->mL[i] * q[(size_t)i * R + r] - dt * bq[r]) + 0.5 * dt * pn;
            }
        }
        free(kq); free(bq);
    }
}

/* ph[node] += Pi^T yhat  (scatter of sensor values to the interpolation nodes) */
static void inject(const oproblem *P, int R, const double *yh, double *ph) {
    for (int s = 0; s < P->n_obs; ++s)
        for (int k = 0; k < 4; ++k)
            for (int r = 0; r < R; ++r)
                ph[(size_t)P->snode[4 * s + k] * R + r] += P->sw[4 * s + k] * yh[(size_t)s * R + r];
}

/* Transpose map: G^T yhat = J^T A^T zhat^1 with zhat^{N_T} = Pi^T yhat^{N_T},
 * zhat^n = Pi^T yhat^n + A^T zhat^{n+1}.  yhat [N_T][n_obs][R]; p [N][R]. */
void orc_adjoint(const oproblem *P, int R, const double *yhat, double *p) {
    const size_t NR = (size_t)P->n_nodes * R;
    double *vh = calloc(NR, sizeof(double)), *w = malloc(sizeof(double) * NR);
    memset(p, 0, sizeof(double) * NR);
    for (int n = P->n_steps; n >= 1; --n) {
        inject(P, R, yhat + (size_t)(n - 1) * P->n_obs * R, p);
        orc_step_transpose(P, R, p, vh, w);
    }
    free(vh); free(w);
}

/* ------------------------------------------------------------------ */
/* The same sweeps with float32 state and arithmetic (test use only)   */
/* ------------------------------------------------------------------ */

/* These repeat orc_forward / orc_adjoint with every stored value (state, matrix
 * entries, masses, dt) rounded to float32 and float32 arithmetic.  They measure
 * the rounding floor of a float32-state implementation of the method, against
 * which a float32 GPU path can be judged where the float64 results are poorly
 * conditioned; they are not used to produce any expected value. */
static inline void row_product_f32(const ocsr *A, int i, int R, const float *restrict x, float *restrict acc) {
    for (int r = 0; r < R; ++r) acc[r] = 0.0f;
    for (int64_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k) {
        const float a = (float)A->val[k];
        const float *xj = x + (size_t)A->col[k] * R;
        for (int r = 0; r < R; ++r) acc[r] += a * xj[r];
    }
}

static void step_f32(const oproblem *P, int R, float *p, float *v, float *ph, float *vn) {
    const int N = P->n_nodes;
    const float dt = (float)P->dt, hdt = (float)(0.5 * P->dt);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < N; ++i)
        for (int r = 0; r < R; ++r) ph[(size_t)i * R + r] = p[(size_t)i * R + r] + hdt * v[(size_t)i * R + r];
#pragma omp parallel
    {
        float *kp = malloc(sizeof(float) * (size_t)R), *bv = malloc(sizeof(float) * (size_t)R);
#pragma omp for schedule(static)
        for (int i = 0; i < N; ++i) {
            const float m = (float)P->mL[i];
            row_product_f32(&P->K, i, R, ph, kp);
            row_product_f32(&P->B, i, R, v, bv);
            for (int r = 0; r < R; ++r) vn[(size_t)i * R + r] = (m * v[(size_t)i * R + r] - dt * kp[r] - dt * bv[r]) / m;
        }
        free(kp); free(bv);
    }
#pragma omp parallel for schedule(static)
    for (int i = 0; i < N; ++i)
        for (int r = 0; r < R; ++r) {
            v[(size_t)i * R + r] = vn[(size_t)i * R + r];
            p[(size_t)i * R + r] = ph[(size_t)i * R + r] + hdt * vn[(size_t)i * R + r];
        }
}

void orc_forward_f32(const oproblem *P, int R, const float *p0, float *y) {
    const size_t NR = (size_t)P->n_nodes * R;
    float *p = malloc(sizeof(float) * NR), *v = calloc(NR, sizeof(float));
    float *ph = malloc(sizeof(float) * NR), *vn = malloc(sizeof(float) * NR);
    memcpy(p, p0, sizeof(float) * NR);
    for (int n = 1; n <= P->n_steps; ++n) {
        step_f32(P, R, p, v, ph, vn);
        float *yn = y + (size_t)(n - 1) * P->n_obs * R;
        for (int s = 0; s < P->n_obs; ++s)
            for (int r = 0; r < R; ++r) {
                float acc = 0.0f;
                for (int k = 0; k < 4; ++k) acc += (float)P->sw[4 * s + k] * p[(size_t)P->snode[4 * s + k] * R + r];
                yn[(size_t)s * R + r] = acc;
            }
    }
    free(p); free(v); free(ph); free(vn);
}

static void step_transpose_f32(const oproblem *P, int R, float *ph, float *vh, float *q) {
    const int N = P->n_nodes;
    const float dt = (float)P->dt, hdt = (float)(0.5 * P->dt);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < N; ++i)
        for (int r = 0; r < R; ++r)
            q[(size_t)i * R + r] = (vh[(size_t)i * R + r] + hdt * ph[(size_t)i * R + r]) / (float)P->mL[i];
#pragma omp parallel
    {
        float *kq = malloc(sizeof(float) * (size_t)R), *bq = malloc(sizeof(float) * (size_t)R);
#pragma omp for schedule(static)
        for (int i = 0; i < N; ++i) {
            row_product_f32(&P->K, i, R, q, kq);
            row_product_f32(&P->B, i, R, q, bq);
            for (int r = 0; r < R; ++r) {
                const float pn = ph[(size_t)i * R + r] - dt * kq[r];
                ph[(size_t)i * R + r] = pn;
                vh[(size_t)i * R + r] = ((float)P->mL[i] * q[(size_t)i * R + r] - dt * bq[r]) + hdt * pn;
            }
        }
        free(kq); free(bq);
    }
}

void orc_adjoint_f32(const oproblem *P, int R, const float *yhat, float *p) {
    const size_t NR = (size_t)P->n_nodes * R;
    float *vh = calloc(NR, sizeof(float)), *q = malloc(sizeof(float) * NR);
    memset(p, 0, sizeof(float) * NR);
    for (int n = P->n_steps; n >= 1; --n) {
        const float *yh = yhat + (size_t)(n - 1) * P->n_obs * R;
        for (int s = 0; s < P->n_obs; ++s)
            for (int k = 0; k < 4; ++k)
                for (int r = 0; r < R; ++r)
                    p[(size_t)P->snode[4 * s + k] * R + r] += (float)P->sw[4 * s + k] * yh[(size_t)s * R + r];
        step_transpose_f32(P, R, p, vh, q);
    }
    free(vh); free(q);
}

/* ------------------------------------------------------------------ */
/* Extended operator of eq. (extended-matrices) with prior factor L     */
/* ------------------------------------------------------------------ */

/* Prior square root L = M_L^{-1/2} (M_L + a K1), so L^T L = (M_L + a K1) M_L^{-1} (M_L + a K1);
 * a = 0 gives L = M_L^{1/2}, the independent prior of eq. (iid-prior). */
static void prior_apply(const oproblem *P, int R, double a, const double *x, double *y) {
    const int N = P->n_nodes;
    orc_spmv(&P->K1, R, x, y);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < N; ++i)
        for (int r = 0; r < R; ++r)
            y[(size_t)i * R + r] = (P->mL[i] * x[(size_t)i * R + r] + a * y[(size_t)i * R + r]) / sqrt(P->mL[i]);
}

static void prior_apply_transpose(const oproblem *P, int R, double a, const double *x, double *y, double *tmp) {
    const int N = P->n_nodes;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < N; ++i)
        for (int r = 0; r < R; ++r) tmp[(size_t)i * R + r] = x[(size_t)i * R + r] / sqrt(P->mL[i]);
    orc_spmv(&P->K1, R, tmp, y);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < N; ++i)
        for (int r = 0; r < R; ++r)
            y[(size_t)i * R + r] = P->mL[i] * tmp[(size_t)i * R + r] + a * y[(size_t)i * R + r];
}

void orc_prior_apply(const oproblem *P, int R, double a, const double *x, double *y) { prior_apply(P, R, a, x, y); }
void orc_prior_apply_transpose(const oproblem *P, int R, double a, const double *x, double *y) {
    double *tmp = malloc(sizeof(double) * (size_t)P->n_nodes * R);
    prior_apply_transpose(P, R, a, x, y, tmp);
    free(tmp);
}

/* per-RHS sum of squares over m rows (sequential, index order) */
static void sumsq(size_t m, int R, const double *x, double *out) {
    for (int r = 0; r < R; ++r) out[r] = 0.0;
    for (size_t i = 0; i < m; ++i)
        for (int r = 0; r < R; ++r) out[r] += x[i * R + r] * x[i * R + r];
}

/* per-RHS dot product over m rows (sequential, index order) */
static void dotr(size_t m, int R, const double *x, const double *y, double *out) {
    for (int r = 0; r < R; ++r) out[r] = 0.0;
    for (size_t i = 0; i < m; ++i)
        for (int r = 0; r < R; ++r) out[r] += x[i * R + r] * y[i * R + r];
}

/* ------------------------------------------------------------------ */
/* CGLS with full reorthogonalisation, applied to eq. (normal-equations) */
/* ------------------------------------------------------------------ */

/* Solves min_x || G_ext x - b ||_2 for R right-hand sides at once, with a fixed
 * number of iterations, x_0 = 0.  G_ext = [ G / sigma ; L ].
 *   bd [N_T][n_obs][R], bp [N][R]      right-hand side b = (bd, bp)
 *   x  [N][R]                          output
 *   resid [R][n_iter+1] or NULL        ||b - G_ext x_k|| (recursively updated residual)
 * The normal-equation residuals s_k = G_ext^T r_k are mutually orthogonal in exact
 * arithmetic; with reorth != 0 each new s_k is orthogonalised against all earlier
 * normalised ones by classical Gram-Schmidt applied twice.  Returns 0, or -1 if
 * memory could not be allocated. */
int orc_cgls(const oproblem *P, int R, double sigma, double prior_a, int n_iter, int reorth,
             const double *bd, const double *bp, double *x, double *resid, double *diag) {
    const int N = P->n_nodes;
    const size_t NR = (size_t)N * R, MR = (size_t)P->n_steps * P->n_obs * R;
    const size_t M = (size_t)P->n_steps * P->n_obs;
    double *rd = malloc(sizeof(double) * MR), *qd = malloc(sizeof(double) * MR);
    double *rp = malloc(sizeof(double) * NR), *qp = malloc(sizeof(double) * NR);
    double *s = malloc(sizeof(double) * NR), *d = malloc(sizeof(double) * NR), *tmp = malloc(sizeof(double) * NR);
    double *Q = reorth ? malloc(sizeof(double) * NR * (size_t)(n_iter + 1)) : NULL;
    double *gamma = malloc(sizeof(double) * R), *delta = malloc(sizeof(double) * R), *w1 = malloc(sizeof(double) * R),
           *w2 = malloc(sizeof(double) * R);
    double *coef = malloc(sizeof(double) * (size_t)R * (size_t)(n_iter + 1));
    if (!rd || !qd || !rp || !qp || !s || !d || !tmp || (reorth && !Q) || !gamma || !delta || !w1 || !w2 || !coef) {
        free(rd); free(qd); free(rp); free(qp); free(s); free(d); free(tmp); free(Q);
        free(gamma); free(delta); free(w1); free(w2); free(coef);
        return -1;
    }
    const double isig = 1.0 / sigma;

    memset(x, 0, sizeof(double) * NR);
    memcpy(rd, bd, sizeof(double) * MR);
    memcpy(rp, bp, sizeof(double) * NR);

    /* s_0 = G_ext^T r_0 = sigma^{-1} G^T r_d + L^T r_p */
#define GEXT_T(dst)                                                                  \
    do {                                                                             \
        orc_adjoint(P, R, rd, dst);                                                  \
        prior_apply_transpose(P, R, prior_a, rp, qp, tmp);                           \
        for (size_t i_ = 0; i_ < NR; ++i_) dst[i_] = isig * dst[i_] + qp[i_];        \
    } while (0)

    GEXT_T(s);
    sumsq((size_t)N, R, s, gamma);
    if (resid || diag) {
        sumsq(M, R, rd, w1); sumsq((size_t)N, R, rp, w2);
        for (int r = 0; r < R; ++r) {
            if (resid) resid[(size_t)r * (n_iter + 1)] = sqrt(w1[r] + w2[r]);
            if (diag) {
                diag[((size_t)r * (n_iter + 1)) * 2] = sqrt(w1[r]);
                diag[((size_t)r * (n_iter + 1)) * 2 + 1] = sqrt(w2[r]);
            }
        }
    }
    if (reorth)
        for (size_t i = 0; i < N; ++i)
            for (int r = 0; r < R; ++r) Q[i * R + r] = gamma[r] > 0 ? s[i * R + r] / sqrt(gamma[r]) : 0.0;
    memcpy(d, s, sizeof(double) * NR);

    for (int k = 1; k <= n_iter; ++k) {
        /* q = G_ext d */
        orc_forward(P, R, d, qd);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < (int64_t)MR; ++i) qd[i] = isig * qd[i];
        prior_apply(P, R, prior_a, d, qp);
        sumsq(M, R, qd, w1);
        sumsq((size_t)N, R, qp, w2);
        for (int r = 0; r < R; ++r) delta[r] = w1[r] + w2[r];
        /* alpha = gamma / ||q||^2 ; x += alpha d ; r -= alpha q */
        for (int r = 0; r < R; ++r) w1[r] = delta[r] > 0 ? gamma[r] / delta[r] : 0.0;
#pragma omp parallel for schedule(static)
        for (int i = 0; i < N; ++i)
            for (int r = 0; r < R; ++r) {
                x[(size_t)i * R + r] += w1[r] * d[(size_t)i * R + r];
                rp[(size_t)i * R + r] -= w1[r] * qp[(size_t)i * R + r];
            }
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < (int64_t)M; ++i)
            for (int r = 0; r < R; ++r) rd[i * R + r] -= w1[r] * qd[i * R + r];
        if (resid || diag) {
            double *a1 = delta, *a2 = w2;
            sumsq(M, R, rd, a1); sumsq((size_t)N, R, rp, a2);
            for (int r = 0; r < R; ++r) {
                if (resid) resid[(size_t)r * (n_iter + 1) + k] = sqrt(a1[r] + a2[r]);
                if (diag) {
                    diag[((size_t)r * (n_iter + 1) + k) * 2] = sqrt(a1[r]);
                    diag[((size_t)r * (n_iter + 1) + k) * 2 + 1] = sqrt(a2[r]);
                }
            }
        }
        if (k == n_iter) break;
        /* s = G_ext^T r */
        GEXT_T(s);
        if (reorth) {
            for (int pass = 0; pass < 2; ++pass) {
                /* coefficients c_j = Q_j^T s, j < k, all from the same s */
#pragma omp parallel for schedule(dynamic, 1)
                for (int j = 0; j < k; ++j) dotr(NR / R, R, Q + (size_t)j * NR, s, coef + (size_t)j * R);
                /* s -= sum_j c_j Q_j */
#pragma omp parallel for schedule(static)
                for (int i = 0; i < N; ++i)
                    for (int j = 0; j < k; ++j)
                        for (int r = 0; r < R; ++r)
                            s[(size_t)i * R + r] -= coef[(size_t)j * R + r] * Q[(size_t)j * NR + (size_t)i * R + r];
            }
        }
        sumsq((size_t)N, R, s, w1);
        if (reorth)
            for (size_t i = 0; i < N; ++i)
                for (int r = 0; r < R; ++r)
                    Q[(size_t)k * NR + i * R + r] = w1[r] > 0 ? s[i * R + r] / sqrt(w1[r]) : 0.0;
        /* beta = gamma_new / gamma ; d = s + beta d */
        for (int r = 0; r < R; ++r) {
            w2[r] = gamma[r] > 0 ? w1[r] / gamma[r] : 0.0;
            gamma[r] = w1[r];
        }
#pragma omp parallel for schedule(static)
        for (int i = 0; i < N; ++i)
            for (int r = 0; r < R; ++r) d[(size_t)i * R + r] = s[(size_t)i * R + r] + w2[r] * d[(size_t)i * R + r];
    }
#undef GEXT_T
    free(rd); free(qd); free(rp); free(qp); free(s); free(d); free(tmp); free(Q);
    free(gamma); free(delta); free(w1); free(w2); free(coef);
    return 0;
}

/* ------------------------------------------------------------------ */
/* LSQR (Paige and Saunders' Golub-Kahan bidiagonalisation), the paper's solver */
/* ------------------------------------------------------------------ */

/* Same problem and outputs as orc_cgls.  With reorth != 0 every new right Lanczos
 * vector v is orthogonalised against all earlier ones (classical Gram-Schmidt
 * applied twice) before it is normalised.  The residual r = b - G_ext x is carried
 * alongside through z = G_ext w (diag, resid).  A new alpha or beta below 1e-15
 * times its first value counts as the exact breakdown of the bidiagonalisation
 * (the least-squares solution is reached); it is set to zero, which leaves x
 * unchanged from then on. */
int orc_lsqr(const oproblem *P, int R, double sigma, double prior_a, int n_iter, int reorth,
             const double *bd, const double *bp, double *x, double *resid, double *diag) {
    const int N = P->n_nodes;
    const size_t NR = (size_t)N * R, M = (size_t)P->n_steps * P->n_obs, MR = M * R;
    const double isig = 1.0 / sigma;
    double *ud = malloc(sizeof(double) * MR), *up = malloc(sizeof(double) * NR);
    double *qd = malloc(sizeof(double) * MR), *qp = malloc(sizeof(double) * NR);
    double *zd = malloc(sizeof(double) * MR), *zp = malloc(sizeof(double) * NR);
    double *rd = malloc(sizeof(double) * MR), *rp = malloc(sizeof(double) * NR);
    double *v = malloc(sizeof(double) * NR), *w = malloc(sizeof(double) * NR), *sv = malloc(sizeof(double) * NR);
    double *tmp = malloc(sizeof(double) * NR);
    double *Q = reorth ? malloc(sizeof(double) * NR * (size_t)(n_iter + 1)) : NULL;
    double *coef = malloc(sizeof(double) * (size_t)R * (size_t)(n_iter + 1));
    double *alpha = malloc(sizeof(double) * R), *beta = malloc(sizeof(double) * R), *rhob = malloc(sizeof(double) * R);
    double *phib = malloc(sizeof(double) * R), *zfac = malloc(sizeof(double) * R), *t1 = malloc(sizeof(double) * R);
    double *a1 = malloc(sizeof(double) * R), *a2 = malloc(sizeof(double) * R);
    double *rho = malloc(sizeof(double) * R), *cs = malloc(sizeof(double) * R), *sn = malloc(sizeof(double) * R);
    double *alpha1 = malloc(sizeof(double) * R), *beta1 = malloc(sizeof(double) * R);
    if (!ud || !up || !qd || !qp || !zd || !zp || !rd || !rp || !v || !w || !sv || !tmp || (reorth && !Q) || !coef ||
        !alpha || !beta || !rhob || !phib || !zfac || !t1 || !a1 || !a2 || !rho || !cs || !sn || !alpha1 || !beta1) {
        free(rho); free(cs); free(sn); free(alpha1); free(beta1);
        free(ud); free(up); free(qd); free(qp); free(zd); free(zp); free(rd); free(rp); free(v); free(w); free(sv);
        free(tmp); free(Q); free(coef); free(alpha); free(beta); free(rhob); free(phib); free(zfac); free(t1);
        free(a1); free(a2);
        return -1;
    }
#define DIAG_AT(k)                                                                          \
    do {                                                                                    \
        if (resid || diag) {                                                                \
            sumsq(M, R, rd, a1); sumsq((size_t)N, R, rp, a2);                               \
            for (int r_ = 0; r_ < R; ++r_) {                                                \
                if (resid) resid[(size_t)r_ * (n_iter + 1) + (k)] = sqrt(a1[r_] + a2[r_]);  \
                if (diag) {                                                                 \
                    diag[((size_t)r_ * (n_iter + 1) + (k)) * 2] = sqrt(a1[r_]);             \
                    diag[((size_t)r_ * (n_iter + 1) + (k)) * 2 + 1] = sqrt(a2[r_]);         \
                }                                                                           \
            }                                                                               \
        }                                                                                   \
    } while (0)

    memset(x, 0, sizeof(double) * NR);
    memcpy(rd, bd, sizeof(double) * MR);
    memcpy(rp, bp, sizeof(double) * NR);
    DIAG_AT(0);
    /* beta_1 u_1 = b */
    sumsq(M, R, bd, a1); sumsq((size_t)N, R, bp, a2);
    for (int r = 0; r < R; ++r) {
        beta[r] = beta1[r] = sqrt(a1[r] + a2[r]);
        t1[r] = beta[r] > 0 ? 1.0 / beta[r] : 0.0;
    }
    for (size_t i = 0; i < M; ++i) for (int r = 0; r < R; ++r) ud[i * R + r] = bd[i * R + r] * t1[r];
    for (size_t i = 0; i < (size_t)N; ++i) for (int r = 0; r < R; ++r) up[i * R + r] = bp[i * R + r] * t1[r];
    /* alpha_1 v_1 = G_ext^T u_1 */
    orc_adjoint(P, R, ud, sv);
    prior_apply_transpose(P, R, prior_a, up, qp, tmp);
    for (size_t i = 0; i < NR; ++i) sv[i] = isig * sv[i] + qp[i];
    sumsq((size_t)N, R, sv, a1);
    for (int r = 0; r < R; ++r) {
        alpha[r] = alpha1[r] = sqrt(a1[r]);
        t1[r] = alpha[r] > 0 ? 1.0 / alpha[r] : 0.0;
    }
    for (size_t i = 0; i < (size_t)N; ++i)
        for (int r = 0; r < R; ++r) { v[i * R + r] = sv[i * R + r] * t1[r]; w[i * R + r] = v[i * R + r]; }
    if (reorth) memcpy(Q, v, sizeof(double) * NR);
    for (int r = 0; r < R; ++r) { phib[r] = beta[r]; rhob[r] = alpha[r]; zfac[r] = 0.0; }

    for (int k = 1; k <= n_iter; ++k) {
        /* q = G_ext v_k ; z_k = q - zfac z_{k-1} (z = G_ext w) */
        orc_forward(P, R, v, qd);
        for (size_t i = 0; i < MR; ++i) qd[i] = isig * qd[i];
        prior_apply(P, R, prior_a, v, qp);
        for (size_t i = 0; i < M; ++i) for (int r = 0; r < R; ++r) zd[i * R + r] = qd[i * R + r] - zfac[r] * (k > 1 ? zd[i * R + r] : 0.0);
        for (size_t i = 0; i < (size_t)N; ++i) for (int r = 0; r < R; ++r) zp[i * R + r] = qp[i * R + r] - zfac[r] * (k > 1 ? zp[i * R + r] : 0.0);
        /* beta_{k+1} u_{k+1} = q - alpha_k u_k */
        for (size_t i = 0; i < M; ++i) for (int r = 0; r < R; ++r) ud[i * R + r] = qd[i * R + r] - alpha[r] * ud[i * R + r];
        for (size_t i = 0; i < (size_t)N; ++i) for (int r = 0; r < R; ++r) up[i * R + r] = qp[i * R + r] - alpha[r] * up[i * R + r];
        sumsq(M, R, ud, a1); sumsq((size_t)N, R, up, a2);
        for (int r = 0; r < R; ++r) {
            beta[r] = sqrt(a1[r] + a2[r]);
            if (!(beta[r] > 1e-15 * beta1[r])) beta[r] = 0.0;
            t1[r] = beta[r] > 0 ? 1.0 / beta[r] : 0.0;
        }
        for (size_t i = 0; i < M; ++i) for (int r = 0; r < R; ++r) ud[i * R + r] *= t1[r];
        for (size_t i = 0; i < (size_t)N; ++i) for (int r = 0; r < R; ++r) up[i * R + r] *= t1[r];
        /* plane rotation: rho_k, c_k, s_k; phi_k; x_k = x_{k-1} + (phi/rho) w_k ; r_k = r_{k-1} - (phi/rho) z_k */
        for (int r = 0; r < R; ++r) {
            rho[r] = sqrt(rhob[r] * rhob[r] + beta[r] * beta[r]);
            cs[r] = rho[r] > 0 ? rhob[r] / rho[r] : 1.0;
            sn[r] = rho[r] > 0 ? beta[r] / rho[r] : 0.0;
            const double phi = cs[r] * phib[r];
            phib[r] = sn[r] * phib[r];
            t1[r] = rho[r] > 0 ? phi / rho[r] : 0.0;
        }
        for (size_t i = 0; i < (size_t)N; ++i)
            for (int r = 0; r < R; ++r) { x[i * R + r] += t1[r] * w[i * R + r]; rp[i * R + r] -= t1[r] * zp[i * R + r]; }
        for (size_t i = 0; i < M; ++i) for (int r = 0; r < R; ++r) rd[i * R + r] -= t1[r] * zd[i * R + r];
        DIAG_AT(k);
        if (k == n_iter) break;
        /* alpha_{k+1} v_{k+1} = G_ext^T u_{k+1} - beta_{k+1} v_k, reorthogonalised */
        orc_adjoint(P, R, ud, sv);
        prior_apply_transpose(P, R, prior_a, up, qp, tmp);
        for (size_t i = 0; i < (size_t)N; ++i)
            for (int r = 0; r < R; ++r) sv[i * R + r] = isig * sv[i * R + r] + qp[i * R + r] - beta[r] * v[i * R + r];
        if (reorth) {
            for (int pass = 0; pass < 2; ++pass) {
#pragma omp parallel for schedule(dynamic, 1)
                for (int j = 0; j < k; ++j) dotr((size_t)N, R, Q + (size_t)j * NR, sv, coef + (size_t)j * R);
#pragma omp parallel for schedule(static)
                for (int i = 0; i < N; ++i)
                    for (int j = 0; j < k; ++j)
                        for (int r = 0; r < R; ++r)
                            sv[(size_t)i * R + r] -= coef[(size_t)j * R + r] * Q[(size_t)j * NR + (size_t)i * R + r];
            }
        }
        sumsq((size_t)N, R, sv, a1);
        for (int r = 0; r < R; ++r) {
            alpha[r] = sqrt(a1[r]);
            if (!(alpha[r] > 1e-15 * alpha1[r])) alpha[r] = 0.0;
            const double theta = sn[r] * alpha[r];            /* theta_{k+1} = s_k alpha_{k+1} */
            rhob[r] = -cs[r] * alpha[r];                      /* rho_bar_{k+1} = -c_k alpha_{k+1} */
            zfac[r] = rho[r] > 0 ? theta / rho[r] : 0.0;      /* theta_{k+1} / rho_k */
            t1[r] = alpha[r] > 0 ? 1.0 / alpha[r] : 0.0;
        }
        for (size_t i = 0; i < (size_t)N; ++i)
            for (int r = 0; r < R; ++r) {
                v[i * R + r] = sv[i * R + r] * t1[r];
                w[i * R + r] = v[i * R + r] - zfac[r] * w[i * R + r];
            }
        if (reorth) memcpy(Q + (size_t)k * NR, v, sizeof(double) * NR);
    }
#undef DIAG_AT
    free(ud); free(up); free(qd); free(qp); free(zd); free(zp); free(rd); free(rp); free(v); free(w); free(sv);
    free(tmp); free(Q); free(coef); free(alpha); free(beta); free(rhob); free(phib); free(zfac); free(t1);
    free(a1); free(a2); free(rho); free(cs); free(sn); free(alpha1); free(beta1);
    return 0;
}

/* ------------------------------------------------------------------ */
/* RTO samples, Algorithm 1 with the right-hand side of eq. (extended-matrices) */
/* ------------------------------------------------------------------ */

/* S posterior samples at once.  The perturbed problem is
 *   min_p sigma^{-2} ||G p - (y + sigma eta)||^2 + ||L (p - p_prior)||^2,
 * p_prior = L^{-1} xi, so b = ( (y + sigma eta)/sigma ; L p_prior ) = ( y/sigma + eta ; xi ).
 *   yobs [N_T][n_obs]; eta [N_T][n_obs][S]; xi [N][S]; samples [N][S]. */
int orc_rto(const oproblem *P, int S, const double *yobs, double sigma, double prior_a, int n_iter, int reorth,
            const double *eta, const double *xi, double *samples, double *resid, int solver, double *diag) {
    const size_t M = (size_t)P->n_steps * P->n_obs;
    double *bd = malloc(sizeof(double) * M * S);
    if (!bd) return -1;
    for (size_t i = 0; i < M; ++i)
        for (int r = 0; r < S; ++r) bd[i * S + r] = yobs[i] / sigma + eta[i * S + r];
    int rc = solver == 1 ? orc_lsqr(P, S, sigma, prior_a, n_iter, reorth, bd, xi, samples, resid, diag)
                         : orc_cgls(P, S, sigma, prior_a, n_iter, reorth, bd, xi, samples, resid, diag);
    free(bd);
    return rc;
}

/* Pointwise mean and standard deviation (1/(S-1) normalisation) of samples [N][S]. */
void orc_stats(int N, int S, const double *samples, double *mean, double *std) {
    for (int i = 0; i < N; ++i) {
        double m = 0.0;
        for (int r = 0; r < S; ++r) m += samples[(size_t)i * S + r];
        m /= S;
        double v = 0.0;
        for (int r = 0; r < S; ++r) {
            double d = samples[(size_t)i * S + r] - m;
            v += d * d;
        }
        mean[i] = m;
        std[i] = S > 1 ? sqrt(v / (S - 1)) : 0.0;
    }
}

/* ------------------------------------------------------------------ */
/* Counter-based standard normals                                        */
/* ------------------------------------------------------------------ */

/* Philox4x64-10 block cipher of Salmon et al. (SC'11): ten rounds of two
 * 64x64 -> 128-bit products (multipliers 0xD2E7470EE14C6C93 on word 0 and
 * 0xCA5A826395121157 on word 2), the high halves xored with the other two words
 * and the round key, the key advanced by the Weyl increments 0x9E3779B97F4A7C15
 * and 0xBB67AE8584CAA73B between rounds. */
void orc_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B97F4A7C15ULL;
            k1 += 0xBB67AE8584CAA73BULL;
        }
        const unsigned __int128 p0 = (unsigned __int128)0xD2E7470EE14C6C93ULL * c0;
        const unsigned __int128 p1 = (unsigned __int128)0xCA5A826395121157ULL * c2;
        const uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        const uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Standard normal number j of stream (seed, kind, k): kind 0 = data
 * perturbation eta_k (j = t*N_obs + s), kind 1 = prior perturbation xi_k (j = node).
 * Block j/4 of the cipher with counter (j/4, k, kind, 0) and key (seed, 0) gives
 * four 64-bit words; words (0, 1) and (2, 3) are two Box-Muller pairs: with
 * U(x) = (x >> 11) 2^-53 in [0, 1), u1 = 1 - U(first) in (0, 1], u2 = U(second),
 * the pair is sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2). */
static double normal_at(uint64_t seed, int kind, int64_t k, int64_t j) {
    const uint64_t ctr[4] = {(uint64_t)j / 4, (uint64_t)k, (uint64_t)kind, 0};
    const uint64_t key[2] = {seed, 0};
    uint64_t w[4];
    orc_philox4x64(ctr, key, w);
    const int lane = (int)(j % 4), pair = lane / 2;
    const double u1 = 1.0 - (double)(w[2 * pair] >> 11) * 0x1p-53;
    const double u2 = (double)(w[2 * pair + 1] >> 11) * 0x1p-53;
    const double rad = sqrt(-2.0 * log(u1));
    const double ang = 6.283185307179586476925286766559 * u2; /* 2 pi */
    return (lane % 2 == 0) ? rad * cos(ang) : rad * sin(ang);
}

/* out[s*len + j] = normal j of stream (seed, kind, k0 + s), s < S, j < len. */
void orc_normals(uint64_t seed, int kind, int64_t k0, int64_t S, int64_t len, double *out) {
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < S; ++s)
        for (int64_t j = 0; j < len; ++j) out[s * len + j] = normal_at(seed, kind, k0 + s, j);
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
