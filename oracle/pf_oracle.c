/*
 * CPU oracle for graph-based Newton-Raphson AC power flow
 * (Shi, Liu, Dai, Wu, Yuan, Wang: "Graph Based Power Flow Calculation for
 * Energy Management System", arXiv 1811.02512).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this file's library.  It shares
 * no code with the GPU library: it is written plainly, sequentially and in
 * fp64, so that each step can be checked against the paper by eye.
 *
 * Contents (each function cites the passage it follows):
 *   - admittance matrix (Sec. III-A, FormMatrixA), pi-model per branch;
 *   - bus injections and mismatch (Sec. II-A: nodal-parallel injection,
 *     mismatch and convergence check), textbook polar form;
 *   - dense Newton-Raphson with a reduced Jacobian and Gaussian elimination
 *     with partial pivoting: the plain definition of the NR solution
 *     (Sec. III, Newton-Raphson linearisation);
 *   - the paper's sparse path: exact minimum-degree ordering (the paper gives
 *     none; our reading), FormFilledGraph (Sec. II-B-1), FormEliminationTree
 *     (Sec. II-B-2), FormHierarchicalPartition (Sec. II-B-2, Table I),
 *     FactorizeGraphA right-looking LDU over the partition (Sec. III-B,
 *     eqs. 1-3), forward substitution, normalisation (eq. 4) and backward
 *     substitution (Sec. III-C);
 *   - a dense adjoint of the converged solution (beyond the paper);
 *   - fast decoupled power flow (Sec. III, Table III; XB matrices, our
 *     reading) on the symmetric factorisation of eqs. 1-3 with scalar
 *     elements, and branch flows of a solved state.
 *
 * Parity pins live in the CPU tests: a 2-bus closed form, power balance
 * (Tellegen) at arbitrary voltages, finite-difference Jacobians, brute-force
 * boolean elimination, Table I's level partition, dense solves checked
 * against LAPACK, and finite differences of the solution for the adjoint.
 *
 * Conventions: buses 0..n-1, per-unit, radians.  Bus types 1 = PQ, 2 = PV,
 * 3 = slack.  A 2x2 block is stored row-major [r0c0, r0c1, r1c0, r1c1]; the
 * row is the equation (0: P, 1: Q for PQ / |V| for PV) and the column is the
 * unknown (0: angle, 1: magnitude).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_PQ 1
#define OR_PV 2
#define OR_SLACK 3

/* ------------------------------------------------------------------------ */
/* Admittance matrix (FormMatrixA, Sec. III-A: admittances on the edges,     */
/* shunts on the vertices).  Every bus i starts its diagonal with its own    */
/* shunt y_sh,i = gsh[i] + j bsh[i] (gsh, bsh may be NULL: no shunts).       */
/* Branch e between f and t with series admittance y = 1/(r + jx) and total  */
/* charging b adds y + jb/2 to both diagonals and -y to both off-diagonals. */
/* Parallel branches are summed.  Output is CSR with sorted columns and an  */
/* explicit diagonal in every row; returns nnz, or -1 on bad input.         */
/* ------------------------------------------------------------------------ */
typedef struct {
    int row, col, br;
    double g, b;
} or_coo;

static int coo_cmp(const void* a, const void* b)
{
    const or_coo* x = (const or_coo*)a;
    const or_coo* y = (const or_coo*)b;
    if (x->row != y->row) return x->row < y->row ? -1 : 1;
    if (x->col != y->col) return x->col < y->col ? -1 : 1;
    if (x->br != y->br) return x->br < y->br ? -1 : 1;
    return 0;
}

int or_ybus(int n, int m, const int32_t* f, const int32_t* t, const double* r,
            const double* x, const double* bc, const double* gsh, const double* bsh,
            int32_t* rowptr, int32_t* col, double* G, double* B)
{
    int cap = n + 4 * m, cnt = 0;
    or_coo* c = (or_coo*)malloc(sizeof(or_coo) * (size_t)(cap > 0 ? cap : 1));
    if (!c) return -1;
    for (int i = 0; i < n; ++i) {
        or_coo z = {i, i, -1, gsh ? gsh[i] : 0.0, bsh ? bsh[i] : 0.0};
        c[cnt++] = z;
    }
    for (int e = 0; e < m; ++e) {
        int a = f[e], b = t[e];
        if (a < 0 || a >= n || b < 0 || b >= n || a == b) {
            free(c);
            return -1;
        }
        double complex y = 1.0 / (r[e] + I * x[e]);
        double complex ysh = I * (bc[e] / 2.0);
        double complex d = y + ysh;
        or_coo e1 = {a, a, e, creal(d), cimag(d)};
        or_coo e2 = {b, b, e, creal(d), cimag(d)};
        or_coo e3 = {a, b, e, -creal(y), -cimag(y)};
        or_coo e4 = {b, a, e, -creal(y), -cimag(y)};
        c[cnt++] = e1;
        c[cnt++] = e2;
        c[cnt++] = e3;
        c[cnt++] = e4;
    }
    qsort(c, (size_t)cnt, sizeof(or_coo), coo_cmp);
    int nnz = 0;
    for (int i = 0; i <= n; ++i) rowptr[i] = 0;
    for (int k = 0; k < cnt; ++k) {
        if (nnz > 0 && col[nnz - 1] == c[k].col && k > 0 && c[k - 1].row == c[k].row) {
            G[nnz - 1] += c[k].g;
            B[nnz - 1] += c[k].b;
        } else {
            col[nnz] = c[k].col;
            G[nnz] = c[k].g;
            B[nnz] = c[k].b;
            rowptr[c[k].row + 1]++;
            nnz++;
        }
    }
    for (int i = 0; i < n; ++i) rowptr[i + 1] += rowptr[i];
    free(c);
    return nnz;
}

/* ------------------------------------------------------------------------ */
/* Injections (Sec. II-A, nodal parallel): textbook polar form               */
/*   P_i = sum_k |V_i||V_k| (G_ik cos t_ik + B_ik sin t_ik)                  */
/*   Q_i = sum_k |V_i||V_k| (G_ik sin t_ik - B_ik cos t_ik),  t_ik = t_i-t_k */
/* ------------------------------------------------------------------------ */
void or_injections(int n, const int32_t* rowptr, const int32_t* col, const double* G,
                   const double* B, const double* Vm, const double* Va, double* P,
                   double* Q)
{
    for (int i = 0; i < n; ++i) {
        double p = 0.0, q = 0.0;
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            int j = col[k];
            double th = Va[i] - Va[j];
            double vv = Vm[i] * Vm[j];
            p += vv * (G[k] * cos(th) + B[k] * sin(th));
            q += vv * (G[k] * sin(th) - B[k] * cos(th));
        }
        P[i] = p;
        Q[i] = q;
    }
}

/* Mismatch F = calculated - scheduled: P at PV and PQ buses, Q at PQ buses. */
/* Returns the infinity norm over those entries (NaN propagates).            */
double or_mismatch(int n, const int8_t* type, const double* P, const double* Q,
                   const double* Psp, const double* Qsp, double* FP, double* FQ)
{
    double nrm = 0.0;
    int bad = 0;
    for (int i = 0; i < n; ++i) {
        FP[i] = 0.0;
        FQ[i] = 0.0;
        if (type[i] == OR_SLACK) continue;
        FP[i] = P[i] - Psp[i];
        if (type[i] == OR_PQ) FQ[i] = Q[i] - Qsp[i];
        double a = fabs(FP[i]), b = fabs(FQ[i]);
        if (!(a == a) || !(b == b)) bad = 1;
        if (a > nrm) nrm = a;
        if (b > nrm) nrm = b;
    }
    return bad ? NAN : nrm;
}

/* ------------------------------------------------------------------------ */
/* Dense Gaussian elimination with partial pivoting: solves A x = rhs,       */
/* A row-major N x N (destroyed), rhs overwritten with x.  Returns 0 or -1   */
/* (singular).                                                               */
/* ------------------------------------------------------------------------ */
int or_dense_solve(int N, double* A, double* rhs)
{
    for (int c = 0; c < N; ++c) {
        int piv = c;
        double best = fabs(A[(size_t)c * N + c]);
        for (int r = c + 1; r < N; ++r) {
            double v = fabs(A[(size_t)r * N + c]);
            if (v > best) {
                best = v;
                piv = r;
            }
        }
        if (best == 0.0 || !(best == best)) return -1;
        if (piv != c) {
            for (int k = 0; k < N; ++k) {
                double tmp = A[(size_t)c * N + k];
                A[(size_t)c * N + k] = A[(size_t)piv * N + k];
                A[(size_t)piv * N + k] = tmp;
            }
            double tmp = rhs[c];
            rhs[c] = rhs[piv];
            rhs[piv] = tmp;
        }
        double d = A[(size_t)c * N + c];
        for (int r = c + 1; r < N; ++r) {
            double l = A[(size_t)r * N + c] / d;
            if (l == 0.0) continue;
            for (int k = c; k < N; ++k) A[(size_t)r * N + k] -= l * A[(size_t)c * N + k];
            rhs[r] -= l * rhs[c];
        }
    }
    for (int c = N - 1; c >= 0; --c) {
        double s = rhs[c];
        for (int k = c + 1; k < N; ++k) s -= A[(size_t)c * N + k] * rhs[k];
        rhs[c] = s / A[(size_t)c * N + c];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Reduced dense Jacobian (the plain definition of the NR linearisation).    */
/* Unknowns: angle of every non-slack bus (ascending bus order), then |V| of */
/* every PQ bus.  Equations: P of every non-slack bus, then Q of every PQ    */
/* bus, in the same orders.  idx_a[bus] / idx_v[bus] give the positions      */
/* (-1 if absent).  J is (na+nv)^2 row-major.                                */
/* ------------------------------------------------------------------------ */
static void dense_index(int n, const int8_t* type, int* idx_a, int* idx_v, int* na, int* nv)
{
    int a = 0, v = 0;
    for (int i = 0; i < n; ++i) idx_a[i] = (type[i] != OR_SLACK) ? a++ : -1;
    for (int i = 0; i < n; ++i) idx_v[i] = (type[i] == OR_PQ) ? a + v++ : -1;
    *na = a;
    *nv = v;
}

/* dP_i/dt_k, dP_i/dV_k, dQ_i/dt_k, dQ_i/dV_k for one Y entry (i, k).        */
static void polar_partials(int i, int k, double Gik, double Bik, const double* Vm,
                           const double* Va, const double* P, const double* Q,
                           double out[4])
{
    if (i != k) {
        double th = Va[i] - Va[k];
        double c = cos(th), s = sin(th);
        out[0] = Vm[i] * Vm[k] * (Gik * s - Bik * c);
        out[1] = Vm[i] * (Gik * c + Bik * s);
        out[2] = -Vm[i] * Vm[k] * (Gik * c + Bik * s);
        out[3] = Vm[i] * (Gik * s - Bik * c);
    } else {
        double v = Vm[i];
        out[0] = -Q[i] - Bik * v * v;
        out[1] = P[i] / v + Gik * v;
        out[2] = P[i] - Gik * v * v;
        out[3] = Q[i] / v - Bik * v;
    }
}

int or_dense_jacobian(int n, const int32_t* rowptr, const int32_t* col, const double* G,
                      const double* B, const int8_t* type, const double* Vm,
                      const double* Va, const double* P, const double* Q, double* J)
{
    int* ia = (int*)malloc(sizeof(int) * (size_t)n);
    int* iv = (int*)malloc(sizeof(int) * (size_t)n);
    int na, nv;
    dense_index(n, type, ia, iv, &na, &nv);
    int N = na + nv;
    memset(J, 0, sizeof(double) * (size_t)N * (size_t)N);
    for (int i = 0; i < n; ++i) {
        if (type[i] == OR_SLACK) continue;
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            int k = col[p];
            if (type[k] == OR_SLACK) continue;
            double d[4];
            polar_partials(i, k, G[p], B[p], Vm, Va, P, Q, d);
            J[(size_t)ia[i] * N + ia[k]] += d[0];
            if (iv[k] >= 0) J[(size_t)ia[i] * N + iv[k]] += d[1];
            if (iv[i] >= 0) {
                J[(size_t)iv[i] * N + ia[k]] += d[2];
                if (iv[k] >= 0) J[(size_t)iv[i] * N + iv[k]] += d[3];
            }
        }
    }
    free(ia);
    free(iv);
    return N;
}

/* Dense NR: the plain definition.  Vm, Va in/out (start values in, solution */
/* out).  Stops when the mismatch norm is below tol at the top of an         */
/* iteration.  Returns 0 converged, 6 not converged, 5 singular, 7 NaN.      */
int or_newton_dense(int n, const int32_t* rowptr, const int32_t* col, const double* G,
                    const double* B, const int8_t* type, const double* Psp,
                    const double* Qsp, double* Vm, double* Va, double tol, int max_iter,
                    int32_t* iters, double* norm)
{
    int* ia = (int*)malloc(sizeof(int) * (size_t)n);
    int* iv = (int*)malloc(sizeof(int) * (size_t)n);
    int na, nv;
    dense_index(n, type, ia, iv, &na, &nv);
    int N = na + nv;
    double* P = (double*)malloc(sizeof(double) * (size_t)n * 4);
    double *Q = P + n, *FP = P + 2 * n, *FQ = P + 3 * n;
    double* J = (double*)malloc(sizeof(double) * (size_t)N * (size_t)N + 8);
    double* rhs = (double*)malloc(sizeof(double) * (size_t)(N + 1));
    int status = 6, it = 0;
    double nrm = 0.0;
    for (;;) {
        or_injections(n, rowptr, col, G, B, Vm, Va, P, Q);
        nrm = or_mismatch(n, type, P, Q, Psp, Qsp, FP, FQ);
        if (!(nrm == nrm) || isinf(nrm)) {
            status = 7;
            break;
        }
        if (nrm < tol) {
            status = 0;
            break;
        }
        if (it >= max_iter) {
            status = 6;
            break;
        }
        or_dense_jacobian(n, rowptr, col, G, B, type, Vm, Va, P, Q, J);
        for (int i = 0; i < n; ++i) {
            if (ia[i] >= 0) rhs[ia[i]] = FP[i];
            if (iv[i] >= 0) rhs[iv[i]] = FQ[i];
        }
        if (or_dense_solve(N, J, rhs) != 0) {
            status = 5;
            break;
        }
        for (int i = 0; i < n; ++i) {
            if (ia[i] >= 0) Va[i] -= rhs[ia[i]];
            if (iv[i] >= 0) Vm[i] -= rhs[iv[i]];
        }
        ++it;
    }
    *iters = it;
    *norm = nrm;
    free(ia);
    free(iv);
    free(P);
    free(J);
    free(rhs);
    return status;
}

/* ======================================================================== */
/* Sparse path, following the paper's steps.                                */
/* The reduced system has one node per non-slack bus, with 2x2 blocks.      */
/* ======================================================================== */

typedef struct {
    int n, nn, slack;
    int32_t* bus_of;   /* nn: bus of reduced node (ascending bus order)   */
    int32_t* node_of;  /* n : reduced node of bus, -1 for the slack       */
    int32_t* perm;     /* nn: node eliminated at position p               */
    int32_t* iperm;    /* nn: position of node                            */
    int32_t* Lp;       /* nn+1: S(p) = Li[Lp[p]..Lp[p+1]) higher nbrs      */
    int32_t* Li;       /* sorted positions q > p adjacent to p in G+       */
    int64_t nnzL;
    int32_t* parent;   /* nn: elimination-tree parent position, -1 root   */
    int32_t* level;    /* nn: hierarchical level (1-based) of position p  */
    int nlev;
    int32_t* level_ptr;   /* nlev+1 */
    int32_t* level_nodes; /* nn: positions, grouped by level, ascending   */
    int32_t* Rp;       /* nn+1: R(p) = lower neighbours of p in G+        */
    int32_t* Ri;       /* ascending positions j < p with p in S(j)         */
    int32_t* Rslot;    /* slot of p inside S(j), global index into Li     */
} or_sym;

void or_sym_free(or_sym* s)
{
    if (!s) return;
    free(s->bus_of);
    free(s->node_of);
    free(s->perm);
    free(s->iperm);
    free(s->Lp);
    free(s->Li);
    free(s->parent);
    free(s->level);
    free(s->level_ptr);
    free(s->level_nodes);
    free(s->Rp);
    free(s->Ri);
    free(s->Rslot);
    free(s);
}

/* Bit matrix helpers (nn x nn adjacency of the elimination graph). */
typedef struct {
    int nn, words;
    uint64_t* bits;
} bitmat;

static int bm_init(bitmat* m, int nn)
{
    m->nn = nn;
    m->words = (nn + 63) / 64;
    m->bits = (uint64_t*)calloc((size_t)nn * (size_t)m->words + 1, sizeof(uint64_t));
    return m->bits ? 0 : -1;
}
static inline int bm_get(const bitmat* m, int a, int b)
{
    return (int)((m->bits[(size_t)a * m->words + (b >> 6)] >> (b & 63)) & 1u);
}
static inline void bm_set(bitmat* m, int a, int b)
{
    m->bits[(size_t)a * m->words + (b >> 6)] |= (uint64_t)1 << (b & 63);
}
static inline void bm_clr(bitmat* m, int a, int b)
{
    m->bits[(size_t)a * m->words + (b >> 6)] &= ~((uint64_t)1 << (b & 63));
}

/* Exact minimum degree (the paper uses the given numbering; this is our    */
/* reading of a fill-reducing order).  The degree of a node is the number   */
/* of distinct uneliminated neighbours in the current elimination graph,    */
/* fill included.  Ties go to the smallest node index, i.e. the smallest    */
/* original bus number.  Eliminating a node joins all its neighbours        */
/* pairwise.  Writes perm[p] = node eliminated at step p.                   */
static int mindeg_order(const bitmat* adj0, int nn, int32_t* perm)
{
    bitmat a;
    if (bm_init(&a, nn)) return -1;
    memcpy(a.bits, adj0->bits, sizeof(uint64_t) * (size_t)nn * (size_t)a.words);
    int* deg = (int*)calloc((size_t)nn + 1, sizeof(int));
    char* done = (char*)calloc((size_t)nn + 1, 1);
    int* nb = (int*)malloc(sizeof(int) * ((size_t)nn + 1));
    for (int v = 0; v < nn; ++v)
        for (int w = 0; w < a.words; ++w) deg[v] += __builtin_popcountll(a.bits[(size_t)v * a.words + w]);
    for (int step = 0; step < nn; ++step) {
        int best = -1;
        for (int v = 0; v < nn; ++v)
            if (!done[v] && (best < 0 || deg[v] < deg[best])) best = v;
        int p = best;
        perm[step] = p;
        done[p] = 1;
        int cnt = 0;
        for (int v = 0; v < nn; ++v)
            if (bm_get(&a, p, v)) nb[cnt++] = v;
        for (int x = 0; x < cnt; ++x)
            for (int y = x + 1; y < cnt; ++y) {
                int u = nb[x], w = nb[y];
                if (!bm_get(&a, u, w)) {
                    bm_set(&a, u, w);
                    bm_set(&a, w, u);
                    deg[u]++;
                    deg[w]++;
                }
            }
        for (int x = 0; x < cnt; ++x) {
            bm_clr(&a, nb[x], p);
            deg[nb[x]]--;
        }
        for (int v = 0; v < a.words; ++v) a.bits[(size_t)p * a.words + v] = 0;
        deg[p] = 0;
    }
    free(deg);
    free(done);
    free(nb);
    free(a.bits);
    return 0;
}

/* Builds the reduced symbolic structure.  ordering 0 = minimum degree,     */
/* 1 = natural (the given bus numbering, as the paper's loops use).         */
/* Returns NULL on invalid input.                                           */
or_sym* or_analyze(int n, int m, const int32_t* f, const int32_t* t, int slack, int ordering)
{
    if (n < 1 || slack < 0 || slack >= n) return NULL;
    or_sym* s = (or_sym*)calloc(1, sizeof(or_sym));
    s->n = n;
    s->slack = slack;
    s->nn = n - 1;
    int nn = s->nn;
    s->bus_of = (int32_t*)malloc(sizeof(int32_t) * ((size_t)nn + 1));
    s->node_of = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    for (int i = 0, k = 0; i < n; ++i) {
        if (i == slack) {
            s->node_of[i] = -1;
        } else {
            s->node_of[i] = k;
            s->bus_of[k++] = i;
        }
    }
    bitmat g;
    bm_init(&g, nn > 0 ? nn : 1);
    for (int e = 0; e < m; ++e) {
        if (f[e] < 0 || f[e] >= n || t[e] < 0 || t[e] >= n || f[e] == t[e]) {
            free(g.bits);
            or_sym_free(s);
            return NULL;
        }
        int a = s->node_of[f[e]], b = s->node_of[t[e]];
        if (a < 0 || b < 0) continue;
        bm_set(&g, a, b);
        bm_set(&g, b, a);
    }
    s->perm = (int32_t*)malloc(sizeof(int32_t) * ((size_t)nn + 1));
    s->iperm = (int32_t*)malloc(sizeof(int32_t) * ((size_t)nn + 1));
    if (ordering == 1) {
        for (int v = 0; v < nn; ++v) s->perm[v] = v;
    } else {
        mindeg_order(&g, nn, s->perm);
    }
    for (int p = 0; p < nn; ++p) s->iperm[s->perm[p]] = p;

    /* FormFilledGraph (Sec. II-B-1): in elimination order, every pair of    */
    /* higher-numbered neighbours of node i becomes adjacent.  The loop over */
    /* i is sequential; the fill created at i is seen by later nodes.        */
    bitmat h;
    bm_init(&h, nn > 0 ? nn : 1);
    for (int a = 0; a < nn; ++a)
        for (int b = 0; b < nn; ++b)
            if (bm_get(&g, a, b)) bm_set(&h, s->iperm[a], s->iperm[b]);
    free(g.bits);
    s->Lp = (int32_t*)malloc(sizeof(int32_t) * ((size_t)nn + 1));
    int64_t cap = 4 * (int64_t)nn + 16, cnt = 0;
    s->Li = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
    int* hi = (int*)malloc(sizeof(int) * ((size_t)nn + 1));
    for (int i = 0; i < nn; ++i) {
        int c = 0;
        for (int j = i + 1; j < nn; ++j)
            if (bm_get(&h, i, j)) hi[c++] = j;
        for (int x = 0; x < c; ++x)
            for (int y = x + 1; y < c; ++y)
                if (!bm_get(&h, hi[x], hi[y])) {
                    bm_set(&h, hi[x], hi[y]); /* fill-in */
                    bm_set(&h, hi[y], hi[x]);
                }
        s->Lp[i] = (int32_t)cnt;
        if (cnt + c > cap) {
            while (cnt + c > cap) cap *= 2;
            s->Li = (int32_t*)realloc(s->Li, sizeof(int32_t) * (size_t)cap);
        }
        for (int x = 0; x < c; ++x) s->Li[cnt++] = hi[x];
    }
    s->Lp[nn] = (int32_t)cnt;
    s->nnzL = cnt;
    free(hi);
    free(h.bits);

    /* FormEliminationTree (Sec. II-B-2): parent = smallest higher neighbour. */
    s->parent = (int32_t*)malloc(sizeof(int32_t) * ((size_t)nn + 1));
    for (int i = 0; i < nn; ++i) s->parent[i] = (s->Lp[i + 1] > s->Lp[i]) ? s->Li[s->Lp[i]] : -1;

    /* FormHierarchicalPartition (Sec. II-B-2, Table I): in each round every */
    /* current leaf gets the round's level, then all of them are removed.    */
    s->level = (int32_t*)malloc(sizeof(int32_t) * ((size_t)nn + 1));
    int* nchild = (int*)calloc((size_t)nn + 1, sizeof(int));
    char* gone = (char*)calloc((size_t)nn + 1, 1);
    int* leaves = (int*)malloc(sizeof(int) * ((size_t)nn + 1));
    for (int i = 0; i < nn; ++i)
        if (s->parent[i] >= 0) nchild[s->parent[i]]++;
    int remaining = nn, lev = 0;
    while (remaining > 0) {
        ++lev;
        int c = 0;
        for (int i = 0; i < nn; ++i)
            if (!gone[i] && nchild[i] == 0) leaves[c++] = i;
        for (int x = 0; x < c; ++x) {
            int i = leaves[x];
            s->level[i] = lev;
            gone[i] = 1;
            if (s->parent[i] >= 0) nchild[s->parent[i]]--;
        }
        remaining -= c;
    }
    s->nlev = lev;
    s->level_ptr = (int32_t*)calloc((size_t)lev + 2, sizeof(int32_t));
    s->level_nodes = (int32_t*)malloc(sizeof(int32_t) * ((size_t)nn + 1));
    for (int i = 0; i < nn; ++i) s->level_ptr[s->level[i]]++;
    for (int l = 1; l <= lev; ++l) s->level_ptr[l] += s->level_ptr[l - 1];
    {
        int* fillp = (int*)malloc(sizeof(int) * ((size_t)lev + 1));
        for (int l = 0; l < lev; ++l) fillp[l] = s->level_ptr[l];
        for (int i = 0; i < nn; ++i) s->level_nodes[fillp[s->level[i] - 1]++] = i;
        free(fillp);
    }
    free(nchild);
    free(gone);
    free(leaves);

    /* Lower neighbour lists R(p), for pull-form forward substitution. */
    s->Rp = (int32_t*)calloc((size_t)nn + 2, sizeof(int32_t));
    s->Ri = (int32_t*)malloc(sizeof(int32_t) * ((size_t)cnt + 1));
    s->Rslot = (int32_t*)malloc(sizeof(int32_t) * ((size_t)cnt + 1));
    for (int64_t q = 0; q < cnt; ++q) s->Rp[s->Li[q] + 1]++;
    for (int i = 0; i < nn; ++i) s->Rp[i + 1] += s->Rp[i];
    {
        int* fillp = (int*)malloc(sizeof(int) * ((size_t)nn + 1));
        for (int i = 0; i < nn; ++i) fillp[i] = s->Rp[i];
        for (int j = 0; j < nn; ++j)
            for (int q = s->Lp[j]; q < s->Lp[j + 1]; ++q) {
                int i = s->Li[q];
                s->Ri[fillp[i]] = j;
                s->Rslot[fillp[i]] = q;
                fillp[i]++;
            }
        free(fillp);
    }
    return s;
}

void or_sym_sizes(const or_sym* s, int32_t* nn, int64_t* nnzL, int32_t* nlev)
{
    *nn = s->nn;
    *nnzL = s->nnzL;
    *nlev = s->nlev;
}

/* perm: bus of the node eliminated at position p. */
void or_sym_export(const or_sym* s, int32_t* perm_bus, int32_t* parent, int32_t* level,
                   int32_t* level_ptr, int32_t* level_nodes, int32_t* Lp, int32_t* Li)
{
    for (int p = 0; p < s->nn; ++p) perm_bus[p] = s->bus_of[s->perm[p]];
    memcpy(parent, s->parent, sizeof(int32_t) * (size_t)s->nn);
    memcpy(level, s->level, sizeof(int32_t) * (size_t)s->nn);
    memcpy(level_ptr, s->level_ptr, sizeof(int32_t) * ((size_t)s->nlev + 1));
    memcpy(level_nodes, s->level_nodes, sizeof(int32_t) * (size_t)s->nn);
    memcpy(Lp, s->Lp, sizeof(int32_t) * ((size_t)s->nn + 1));
    memcpy(Li, s->Li, sizeof(int32_t) * (size_t)s->nnzL);
}

/* Position of q in S(p) (binary search); -1 if absent. */
static int64_t slot_of(const or_sym* s, int p, int q)
{
    int lo = s->Lp[p], hi = s->Lp[p + 1] - 1;
    while (lo <= hi) {
        int mid = (lo + hi) / 2;
        if (s->Li[mid] == q) return mid;
        if (s->Li[mid] < q) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

/* 2x2 block helpers. */
static void b_mul(const double* a, const double* b, double* c)
{
    c[0] = a[0] * b[0] + a[1] * b[2];
    c[1] = a[0] * b[1] + a[1] * b[3];
    c[2] = a[2] * b[0] + a[3] * b[2];
    c[3] = a[2] * b[1] + a[3] * b[3];
}
static int b_inv(const double* a, double* r)
{
    double det = a[0] * a[3] - a[1] * a[2];
    if (det == 0.0 || !isfinite(det)) return -1;
    r[0] = a[3] / det;
    r[1] = -a[1] / det;
    r[2] = -a[2] / det;
    r[3] = a[0] / det;
    return 0;
}
static void b_mv(const double* a, const double* x, double* y)
{
    y[0] = a[0] * x[0] + a[1] * x[1];
    y[1] = a[2] * x[0] + a[3] * x[1];
}

/* Block Jacobian in the filled layout.  D[p] = diagonal block of position  */
/* p; Lb[q] = block (Li[q], p) below the diagonal, Ub[q] = block (p, Li[q]) */
/* above it, for q in [Lp[p], Lp[p+1]).  Fill positions stay zero.          */
/* PV rows are the |V| equation: the Q-row becomes (0, 1) on the diagonal   */
/* and (0, 0) elsewhere, and the |V| column of a PV bus is zero off its own */
/* row, so the Newton step keeps |V| fixed there (our reading).             */
void or_block_jacobian(const or_sym* s, const int32_t* rowptr, const int32_t* col,
                       const double* G, const double* B, const int8_t* type,
                       const double* Vm, const double* Va, const double* P,
                       const double* Q, double* D, double* Lb, double* Ub)
{
    int nn = s->nn;
    memset(D, 0, sizeof(double) * 4 * (size_t)nn);
    memset(Lb, 0, sizeof(double) * 4 * (size_t)s->nnzL);
    memset(Ub, 0, sizeof(double) * 4 * (size_t)s->nnzL);
    for (int ni = 0; ni < nn; ++ni) {
        int i = s->bus_of[ni];
        int pi = s->iperm[ni];
        for (int a = rowptr[i]; a < rowptr[i + 1]; ++a) {
            int k = col[a];
            int nk = s->node_of[k];
            if (nk < 0) continue;
            int pk = s->iperm[nk];
            double d[4];
            polar_partials(i, k, G[a], B[a], Vm, Va, P, Q, d);
            if (type[i] == OR_PV) {
                d[2] = 0.0;
                d[3] = (i == k) ? 1.0 : 0.0;
            }
            if (type[k] == OR_PV) {
                if (i != k) {
                    d[1] = 0.0;
                    d[3] = 0.0;
                } else {
                    d[1] = 0.0;
                }
            }
            double* dst;
            if (pi == pk) {
                dst = D + 4 * (size_t)pi;
            } else if (pi > pk) {
                dst = Lb + 4 * (size_t)slot_of(s, pk, pi);
            } else {
                dst = Ub + 4 * (size_t)slot_of(s, pi, pk);
            }
            for (int c = 0; c < 4; ++c) dst[c] += d[c];
        }
    }
}

/* FactorizeGraphA (Sec. III-B): partitions 1..p in order, nodes of a       */
/* partition in ascending order.  For node i: D_i = A_ii; the row is        */
/* normalised, U_ij = D_i^-1 A_ij; every intersection (k, j) of the column  */
/* and row structure of i, zero or not, is updated A_kj -= A_ki U_ij (k = j */
/* is the diagonal); finally the column is normalised, L_ki = A_ki D_i^-1.  */
/* In place: D keeps D_i, Lb becomes L, Ub becomes U (unit triangular).     */
/* Returns -1 on success, else the first position whose pivot block is      */
/* singular or non-finite.                                                  */
int or_factor(const or_sym* s, double* D, double* Lb, double* Ub)
{
    double Di[4], Dinv[4], t[4];
    for (int l = 0; l < s->nlev; ++l) {
        for (int x = s->level_ptr[l]; x < s->level_ptr[l + 1]; ++x) {
            int i = s->level_nodes[x];
            memcpy(Di, D + 4 * (size_t)i, sizeof Di);
            if (b_inv(Di, Dinv)) return i;
            for (int q = s->Lp[i]; q < s->Lp[i + 1]; ++q) {
                b_mul(Dinv, Ub + 4 * (size_t)q, t);
                memcpy(Ub + 4 * (size_t)q, t, sizeof t);
            }
            for (int qk = s->Lp[i]; qk < s->Lp[i + 1]; ++qk) {
                int k = s->Li[qk];
                const double* Aki = Lb + 4 * (size_t)qk;
                for (int qj = s->Lp[i]; qj < s->Lp[i + 1]; ++qj) {
                    int j = s->Li[qj];
                    const double* Uij = Ub + 4 * (size_t)qj;
                    double* dst;
                    if (k == j) dst = D + 4 * (size_t)k;
                    else if (k > j) dst = Lb + 4 * (size_t)slot_of(s, j, k);
                    else dst = Ub + 4 * (size_t)slot_of(s, k, j);
                    b_mul(Aki, Uij, t);
                    for (int c = 0; c < 4; ++c) dst[c] -= t[c];
                }
            }
            for (int q = s->Lp[i]; q < s->Lp[i + 1]; ++q) {
                b_mul(Lb + 4 * (size_t)q, Dinv, t);
                memcpy(Lb + 4 * (size_t)q, t, sizeof t);
            }
        }
    }
    return -1;
}

/* Forward substitution (Sec. III-C-1), partitions 1..p:                    */
/*   z_i = b_i - sum_{j < i, L_ij != 0} L_ij z_j;                           */
/* normalisation (eq. 4): y_i = D_i^-1 z_i;                                 */
/* backward substitution (Sec. III-C-3), partitions p..1:                   */
/*   x_i = y_i - sum_{j > i, U_ij != 0} U_ij x_j.                           */
/* rhs (2 per position) is overwritten with x.  Returns 0, or -1 if a       */
/* pivot block is singular.                                                 */
int or_solve(const or_sym* s, const double* D, const double* Lb, const double* Ub,
             double* rhs)
{
    double t[2], Dinv[4];
    for (int l = 0; l < s->nlev; ++l)
        for (int x = s->level_ptr[l]; x < s->level_ptr[l + 1]; ++x) {
            int i = s->level_nodes[x];
            for (int r = s->Rp[i]; r < s->Rp[i + 1]; ++r) {
                int j = s->Ri[r];
                b_mv(Lb + 4 * (size_t)s->Rslot[r], rhs + 2 * (size_t)j, t);
                rhs[2 * i] -= t[0];
                rhs[2 * i + 1] -= t[1];
            }
        }
    for (int i = 0; i < s->nn; ++i) {
        if (b_inv(D + 4 * (size_t)i, Dinv)) return -1;
        b_mv(Dinv, rhs + 2 * (size_t)i, t);
        rhs[2 * i] = t[0];
        rhs[2 * i + 1] = t[1];
    }
    for (int l = s->nlev - 1; l >= 0; --l)
        for (int x = s->level_ptr[l]; x < s->level_ptr[l + 1]; ++x) {
            int i = s->level_nodes[x];
            for (int q = s->Lp[i]; q < s->Lp[i + 1]; ++q) {
                b_mv(Ub + 4 * (size_t)q, rhs + 2 * (size_t)s->Li[q], t);
                rhs[2 * i] -= t[0];
                rhs[2 * i + 1] -= t[1];
            }
        }
    return 0;
}

/* Sparse NR along the paper's path.  Same stopping rule and update as the  */
/* dense version; the rhs of position p is (F_P, F_Q) of its bus (F_Q = 0   */
/* at PV buses) and the step is subtracted.  Returns 0 / 5 (zero pivot, and */
/* *bad_node = position) / 6 / 7 like or_newton_dense.                      */
int or_newton_sparse(const or_sym* s, const int32_t* rowptr, const int32_t* col,
                     const double* G, const double* B, const int8_t* type,
                     const double* Psp, const double* Qsp, double* Vm, double* Va,
                     double tol, int max_iter, int32_t* iters, double* norm,
                     int32_t* bad_node)
{
    int n = s->n, nn = s->nn;
    double* P = (double*)malloc(sizeof(double) * (size_t)n * 4);
    double *Q = P + n, *FP = P + 2 * n, *FQ = P + 3 * n;
    double* D = (double*)malloc(sizeof(double) * 4 * ((size_t)nn + 1));
    double* Lb = (double*)malloc(sizeof(double) * 4 * ((size_t)s->nnzL + 1));
    double* Ub = (double*)malloc(sizeof(double) * 4 * ((size_t)s->nnzL + 1));
    double* rhs = (double*)malloc(sizeof(double) * 2 * ((size_t)nn + 1));
    int status = 6, it = 0;
    double nrm = 0.0;
    *bad_node = -1;
    for (;;) {
        or_injections(n, rowptr, col, G, B, Vm, Va, P, Q);
        nrm = or_mismatch(n, type, P, Q, Psp, Qsp, FP, FQ);
        if (!(nrm == nrm) || isinf(nrm)) {
            status = 7;
            break;
        }
        if (nrm < tol) {
            status = 0;
            break;
        }
        if (it >= max_iter) {
            status = 6;
            break;
        }
        or_block_jacobian(s, rowptr, col, G, B, type, Vm, Va, P, Q, D, Lb, Ub);
        for (int ni = 0; ni < nn; ++ni) {
            int p = s->iperm[ni], bus = s->bus_of[ni];
            rhs[2 * p] = FP[bus];
            rhs[2 * p + 1] = FQ[bus];
        }
        int bad = or_factor(s, D, Lb, Ub);
        if (bad >= 0) {
            *bad_node = bad;
            status = 5;
            break;
        }
        or_solve(s, D, Lb, Ub, rhs);
        for (int ni = 0; ni < nn; ++ni) {
            int p = s->iperm[ni], bus = s->bus_of[ni];
            Va[bus] -= rhs[2 * p];
            if (type[bus] == OR_PQ) Vm[bus] -= rhs[2 * p + 1];
        }
        ++it;
    }
    *iters = it;
    *norm = nrm;
    free(P);
    free(D);
    free(Lb);
    free(Ub);
    free(rhs);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Adjoint of the converged solution (beyond the paper).                     */
/* F(x, p) = 0 defines the state x(p), so with J^T lam = g (g = dL/dx):       */
/*   dL/dPsp_i = lam_P,i (non-slack), dL/dQsp_i = lam_Q,i (PQ),              */
/*   dL/dx_e   = -sum_i lam_i . d(P_i, Q_i)/dx_e, dy_e/dx_e = -j y_e^2.       */
/* lamP/lamQ are per bus (zero where absent).                                */
/* ------------------------------------------------------------------------ */
static void adjoint_param_grads(int n, int m, const int32_t* f, const int32_t* t,
                                const double* r, const double* x, const double* Vm,
                                const double* Va, const double* lamP, const double* lamQ,
                                double* gP, double* gQ, double* gx)
{
    for (int i = 0; i < n; ++i) {
        gP[i] = lamP[i];
        gQ[i] = lamQ[i];
    }
    for (int e = 0; e < m; ++e) {
        int a = f[e], b = t[e];
        double complex z = r[e] + I * x[e];
        double complex y = 1.0 / z;
        double complex dy = -I * y * y;
        double complex Va_ = Vm[a] * cexp(I * Va[a]);
        double complex Vb_ = Vm[b] * cexp(I * Va[b]);
        double complex dSa = Va_ * conj(dy * (Va_ - Vb_));
        double complex dSb = Vb_ * conj(dy * (Vb_ - Va_));
        double acc = 0.0;
        acc += lamP[a] * creal(dSa) + lamQ[a] * cimag(dSa);
        acc += lamP[b] * creal(dSb) + lamQ[b] * cimag(dSb);
        gx[e] = -acc;
    }
}

/* Dense: J^T lam = g by Gaussian elimination on the reduced dense J.        */
/* gVm, gVa: loss gradients per bus (slack and PV |V| entries ignored).      */
/* Returns 0 or 5 (singular).                                                */
int or_adjoint_dense(int n, int m, const int32_t* f, const int32_t* t, const double* r,
                     const double* x, const int32_t* rowptr, const int32_t* col,
                     const double* G, const double* B, const int8_t* type,
                     const double* Vm, const double* Va, const double* gVm,
                     const double* gVa, double* gP, double* gQ, double* gx)
{
    int* ia = (int*)malloc(sizeof(int) * (size_t)n);
    int* iv = (int*)malloc(sizeof(int) * (size_t)n);
    int na, nv;
    dense_index(n, type, ia, iv, &na, &nv);
    int N = na + nv;
    double* P = (double*)malloc(sizeof(double) * 4 * (size_t)n);
    double* Q = P + n;
    double* lP = P + 2 * n;
    double* lQ = P + 3 * n;
    or_injections(n, rowptr, col, G, B, Vm, Va, P, Q);
    double* J = (double*)malloc(sizeof(double) * (size_t)N * (size_t)N + 8);
    double* JT = (double*)malloc(sizeof(double) * (size_t)N * (size_t)N + 8);
    double* lam = (double*)malloc(sizeof(double) * ((size_t)N + 1));
    or_dense_jacobian(n, rowptr, col, G, B, type, Vm, Va, P, Q, J);
    for (int a = 0; a < N; ++a)
        for (int b = 0; b < N; ++b) JT[(size_t)a * N + b] = J[(size_t)b * N + a];
    for (int i = 0; i < n; ++i) {
        if (ia[i] >= 0) lam[ia[i]] = gVa[i];
        if (iv[i] >= 0) lam[iv[i]] = gVm[i];
    }
    int st = or_dense_solve(N, JT, lam) ? 5 : 0;
    for (int i = 0; i < n; ++i) {
        lP[i] = (st == 0 && ia[i] >= 0) ? lam[ia[i]] : 0.0;
        lQ[i] = (st == 0 && iv[i] >= 0) ? lam[iv[i]] : 0.0;
    }
    adjoint_param_grads(n, m, f, t, r, x, Vm, Va, lP, lQ, gP, gQ, gx);
    free(ia);
    free(iv);
    free(P);
    free(J);
    free(JT);
    free(lam);
    return st;
}

/* Transposed solve with the paper-path factors, A^T x = rhs, A = L D U:     */
/*   U^T p = rhs over partitions 1..p: p_i = rhs_i - sum_{j<i} U_ji^T p_j;   */
/*   normalisation q_i = D_i^-T p_i;                                         */
/*   L^T x = q over partitions p..1:   x_i = q_i - sum_{k>i} L_ki^T x_k.     */
int or_solve_transpose(const or_sym* s, const double* D, const double* Lb, const double* Ub,
                       double* rhs)
{
    double Dinv[4];
    for (int l = 0; l < s->nlev; ++l)
        for (int x = s->level_ptr[l]; x < s->level_ptr[l + 1]; ++x) {
            int i = s->level_nodes[x];
            for (int r = s->Rp[i]; r < s->Rp[i + 1]; ++r) {
                const double* U = Ub + 4 * (size_t)s->Rslot[r];
                const double* pj = rhs + 2 * (size_t)s->Ri[r];
                rhs[2 * i] -= U[0] * pj[0] + U[2] * pj[1];
                rhs[2 * i + 1] -= U[1] * pj[0] + U[3] * pj[1];
            }
        }
    for (int i = 0; i < s->nn; ++i) {
        if (b_inv(D + 4 * (size_t)i, Dinv)) return -1;
        double p0 = rhs[2 * i], p1 = rhs[2 * i + 1];
        rhs[2 * i] = Dinv[0] * p0 + Dinv[2] * p1;
        rhs[2 * i + 1] = Dinv[1] * p0 + Dinv[3] * p1;
    }
    for (int l = s->nlev - 1; l >= 0; --l)
        for (int x = s->level_ptr[l]; x < s->level_ptr[l + 1]; ++x) {
            int i = s->level_nodes[x];
            for (int q = s->Lp[i]; q < s->Lp[i + 1]; ++q) {
                const double* L = Lb + 4 * (size_t)q;
                const double* xk = rhs + 2 * (size_t)s->Li[q];
                rhs[2 * i] -= L[0] * xk[0] + L[2] * xk[1];
                rhs[2 * i + 1] -= L[1] * xk[0] + L[3] * xk[1];
            }
        }
    return 0;
}

/* Sparse adjoint along the paper's path: block Jacobian at the state in the */
/* filled layout, FactorizeGraphA, then the transposed solve.  The rhs of    */
/* position p is (dL/dtheta, dL/d|V|) of its bus, with d|V| zero at PV       */
/* buses (|V| fixed there).  Returns 0, or 5 on a zero pivot.                */
int or_adjoint_sparse(const or_sym* s, int m, const int32_t* f, const int32_t* t,
                      const double* r, const double* x, const int32_t* rowptr,
                      const int32_t* col, const double* G, const double* B,
                      const int8_t* type, const double* Vm, const double* Va,
                      const double* gVm, const double* gVa, double* gP, double* gQ,
                      double* gx)
{
    int n = s->n, nn = s->nn;
    double* P = (double*)malloc(sizeof(double) * 4 * (size_t)n);
    double *Q = P + n, *lP = P + 2 * n, *lQ = P + 3 * n;
    double* D = (double*)malloc(sizeof(double) * 4 * ((size_t)nn + 1));
    double* Lb = (double*)malloc(sizeof(double) * 4 * ((size_t)s->nnzL + 1));
    double* Ub = (double*)malloc(sizeof(double) * 4 * ((size_t)s->nnzL + 1));
    double* rhs = (double*)malloc(sizeof(double) * 2 * ((size_t)nn + 1));
    or_injections(n, rowptr, col, G, B, Vm, Va, P, Q);
    or_block_jacobian(s, rowptr, col, G, B, type, Vm, Va, P, Q, D, Lb, Ub);
    int st = 0;
    if (or_factor(s, D, Lb, Ub) >= 0) st = 5;
    for (int ni = 0; ni < nn; ++ni) {
        int p = s->iperm[ni], bus = s->bus_of[ni];
        rhs[2 * p] = gVa[bus];
        rhs[2 * p + 1] = (type[bus] == OR_PV) ? 0.0 : gVm[bus];
    }
    if (st == 0 && or_solve_transpose(s, D, Lb, Ub, rhs)) st = 5;
    for (int i = 0; i < n; ++i) {
        lP[i] = 0.0;
        lQ[i] = 0.0;
    }
    for (int ni = 0; ni < nn && st == 0; ++ni) {
        int p = s->iperm[ni], bus = s->bus_of[ni];
        lP[bus] = rhs[2 * p];
        lQ[bus] = (type[bus] == OR_PV) ? 0.0 : rhs[2 * p + 1];
    }
    adjoint_param_grads(n, m, f, t, r, x, Vm, Va, lP, lQ, gP, gQ, gx);
    free(P);
    free(D);
    free(Lb);
    free(Ub);
    free(rhs);
    return st;
}

/* ======================================================================== */
/* Fast decoupled power flow (Sec. III: the second method the paper runs;   */
/* Table III).  The paper fixes no variant; this follows the XB scheme of   */
/* Stott and Alsac with van Amerongen's choice of matrices (our reading):   */
/*   B'  : branch reactances only, b'_ik = -sum_e 1/x_e over branches (i,k), */
/*         b'_ii = sum_e 1/x_e over branches at i (slack branches included); */
/*   B'' : -Im(Y) of the full pi-model (r, x and charging) and of the bus    */
/*         shunts (bsh, may be NULL), so b''_ii also takes -bsh[i].          */
/* Both are symmetric, so the paper's symmetric factorisation applies       */
/* (Sec. III-B, eqs. 1-3).  Positions and slots are those of or_analyze:     */
/* d[p] diagonal, a[q] = entry (p, Li[q]) = entry (Li[q], p).  B'' keeps    */
/* the non-slack pattern: a PV position gets diagonal 1 and zero off-        */
/* diagonals, which leaves the reduced system over PQ buses unchanged.       */
/* ======================================================================== */
void or_fdpf_matrices(const or_sym* s, int m, const int32_t* f, const int32_t* t,
                      const double* r, const double* x, const double* b, const double* bsh,
                      const int8_t* type, double* d1, double* a1, double* d2, double* a2)
{
    int nn = s->nn;
    memset(d1, 0, sizeof(double) * (size_t)nn);
    memset(d2, 0, sizeof(double) * (size_t)nn);
    memset(a1, 0, sizeof(double) * (size_t)s->nnzL);
    memset(a2, 0, sizeof(double) * (size_t)s->nnzL);
    if (bsh)
        for (int ni = 0; ni < nn; ++ni) d2[s->iperm[ni]] -= bsh[s->bus_of[ni]];
    for (int e = 0; e < m; ++e) {
        int nf = s->node_of[f[e]], nt = s->node_of[t[e]];
        int pf = nf >= 0 ? s->iperm[nf] : -1, pt = nt >= 0 ? s->iperm[nt] : -1;
        double bx = 1.0 / x[e];
        double bs = x[e] / (r[e] * r[e] + x[e] * x[e]); /* -Im(1/(r+jx)) */
        double sh = b[e] / 2.0;
        if (pf >= 0) {
            d1[pf] += bx;
            d2[pf] += bs - sh;
        }
        if (pt >= 0) {
            d1[pt] += bx;
            d2[pt] += bs - sh;
        }
        if (pf >= 0 && pt >= 0) {
            int lo = pf < pt ? pf : pt, hi = pf < pt ? pt : pf;
            int64_t q = slot_of(s, lo, hi);
            a1[q] -= bx;
            a2[q] -= bs;
        }
    }
    for (int ni = 0; ni < nn; ++ni) {
        if (type[s->bus_of[ni]] != OR_PV) continue;
        int p = s->iperm[ni];
        d2[p] = 1.0;
        for (int q = s->Lp[p]; q < s->Lp[p + 1]; ++q) a2[q] = 0.0;
        for (int rr = s->Rp[p]; rr < s->Rp[p + 1]; ++rr) a2[s->Rslot[rr]] = 0.0;
    }
}

/* FactorizeGraphA with scalar elements (Sec. III-B), right-looking over the */
/* partition like or_factor, on a full (non-symmetric) copy so that eq. 2   */
/* can be checked on the result: for i in partition order, the row is      */
/* normalised u_ij = a_ij / a_ii, every intersection of the column and row  */
/* structure is updated a_kj -= a_ki u_ij, then the column is normalised    */
/* l_ki = a_ki / a_ii.  In place: d keeps d_i, lo becomes L, up becomes U.  */
/* Returns -1, or the first position with a zero or non-finite pivot.       */
int or_factor1(const or_sym* s, double* d, double* lo, double* up)
{
    for (int l = 0; l < s->nlev; ++l)
        for (int xx = s->level_ptr[l]; xx < s->level_ptr[l + 1]; ++xx) {
            int i = s->level_nodes[xx];
            double di = d[i];
            if (di == 0.0 || !isfinite(di)) return i;
            for (int q = s->Lp[i]; q < s->Lp[i + 1]; ++q) up[q] /= di;
            for (int qk = s->Lp[i]; qk < s->Lp[i + 1]; ++qk) {
                int k = s->Li[qk];
                for (int qj = s->Lp[i]; qj < s->Lp[i + 1]; ++qj) {
                    int j = s->Li[qj];
                    double v = lo[qk] * up[qj];
                    if (k == j) d[k] -= v;
                    else if (k > j) lo[slot_of(s, j, k)] -= v;
                    else up[slot_of(s, k, j)] -= v;
                }
            }
            for (int q = s->Lp[i]; q < s->Lp[i + 1]; ++q) lo[q] /= di;
        }
    return -1;
}

/* Forward substitution, normalisation (eq. 4) and backward substitution    */
/* (Sec. III-C) with scalar factors; rhs (one per position) is overwritten. */
void or_solve1(const or_sym* s, const double* d, const double* lo, const double* up,
               double* rhs)
{
    for (int l = 0; l < s->nlev; ++l)
        for (int xx = s->level_ptr[l]; xx < s->level_ptr[l + 1]; ++xx) {
            int i = s->level_nodes[xx];
            for (int rr = s->Rp[i]; rr < s->Rp[i + 1]; ++rr)
                rhs[i] -= lo[s->Rslot[rr]] * rhs[s->Ri[rr]];
        }
    for (int i = 0; i < s->nn; ++i) rhs[i] /= d[i];
    for (int l = s->nlev - 1; l >= 0; --l)
        for (int xx = s->level_ptr[l]; xx < s->level_ptr[l + 1]; ++xx) {
            int i = s->level_nodes[xx];
            for (int q = s->Lp[i]; q < s->Lp[i + 1]; ++q) rhs[i] -= up[q] * rhs[s->Li[q]];
        }
}

/* The fast decoupled iteration on factored B' (d1, l1, u1) and B''         */
/* (d2, l2, u2).  F = calculated - scheduled as for NR.  Each iteration:     */
/* stop if max|F| < tol (status 0), else theta -= B'^-1 (F_P / |V|); stop    */
/* if max|F| < tol; else |V| -= B''^-1 (F_Q / |V|) at PQ buses.  iters       */
/* counts the angle half-steps, max_iter bounds them.  Returns 0, 6 (not     */
/* converged) or 7 (non-finite).                                             */
int or_fdpf(const or_sym* s, const int32_t* rowptr, const int32_t* col, const double* G,
            const double* B, const int8_t* type, const double* Psp, const double* Qsp,
            const double* d1, const double* l1, const double* u1, const double* d2,
            const double* l2, const double* u2, double* Vm, double* Va, double tol,
            int max_iter, int32_t* iters, double* norm)
{
    int n = s->n, nn = s->nn;
    double* P = (double*)malloc(sizeof(double) * (size_t)n * 4);
    double *Q = P + n, *FP = P + 2 * n, *FQ = P + 3 * n;
    double* rhs = (double*)malloc(sizeof(double) * ((size_t)nn + 1));
    int status = 6, it = 0, half = 0;
    double nrm = 0.0;
    for (;;) {
        or_injections(n, rowptr, col, G, B, Vm, Va, P, Q);
        nrm = or_mismatch(n, type, P, Q, Psp, Qsp, FP, FQ);
        if (!(nrm == nrm) || isinf(nrm)) {
            status = 7;
            break;
        }
        if (nrm < tol) {
            status = 0;
            break;
        }
        if (half == 0) {
            if (it >= max_iter) {
                status = 6;
                break;
            }
            for (int ni = 0; ni < nn; ++ni) {
                int bus = s->bus_of[ni];
                rhs[s->iperm[ni]] = FP[bus] / Vm[bus];
            }
            or_solve1(s, d1, l1, u1, rhs);
            for (int ni = 0; ni < nn; ++ni) Va[s->bus_of[ni]] -= rhs[s->iperm[ni]];
            ++it;
            half = 1;
        } else {
            for (int ni = 0; ni < nn; ++ni) {
                int bus = s->bus_of[ni];
                rhs[s->iperm[ni]] = type[bus] == OR_PQ ? FQ[bus] / Vm[bus] : 0.0;
            }
            or_solve1(s, d2, l2, u2, rhs);
            for (int ni = 0; ni < nn; ++ni) {
                int bus = s->bus_of[ni];
                if (type[bus] == OR_PQ) Vm[bus] -= rhs[s->iperm[ni]];
            }
            half = 0;
        }
    }
    *iters = it;
    *norm = nrm;
    free(P);
    free(rhs);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Branch flows after convergence (Sec. II-A lists this post-convergence    */
/* step among the nodal-parallel ones).  Branch e from f to t,              */
/* pi-model with series y = 1/(r + jx) and charging b:                      */
/*   I_ft = (y + jb/2) V_f - y V_t,  S_ft = V_f conj(I_ft), and the same    */
/*   with f and t swapped; losses = S_ft + S_tf.                            */
/* ------------------------------------------------------------------------ */
void or_branch_flows(int m, const int32_t* f, const int32_t* t, const double* r,
                     const double* x, const double* b, const double* Vm, const double* Va,
                     double* Pft, double* Qft, double* Ptf, double* Qtf)
{
    for (int e = 0; e < m; ++e) {
        double complex y = 1.0 / (r[e] + I * x[e]);
        double complex ysh = I * (b[e] / 2.0);
        double complex vf = Vm[f[e]] * cexp(I * Va[f[e]]);
        double complex vt = Vm[t[e]] * cexp(I * Va[t[e]]);
        double complex sft = vf * conj((y + ysh) * vf - y * vt);
        double complex stf = vt * conj((y + ysh) * vt - y * vf);
        Pft[e] = creal(sft);
        Qft[e] = cimag(sft);
        Ptf[e] = creal(stf);
        Qtf[e] = cimag(stf);
    }
}
