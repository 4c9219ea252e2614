// libpf: HIP kernels for gfx950 and the C ABI declared in include/pf.h.
//
// Kernel map (paper sections in brackets):
//   k_ybus        FormMatrixA, one thread per (case, bus row)      [III-A]
//   k_mismatch    injections, mismatch, max-norm, one WG per case  [II-A]
//   k_jacobian    Jacobian blocks into the filled layout            [III]
//   k_factor      FactorizeGraphA, level by level, one WG per case  [III-B]
//   k_solve       forward / normalisation / backward substitution  [III-C]
//   k_newton      the whole Newton loop of one case per workgroup   [III]
//   k_adj_*       adjoint parameter gradients (beyond the paper)
//
// Work decomposition inside a workgroup: hierarchical levels run one after
// the other with a workgroup barrier between them; inside a level, each
// node gets a group of g lanes (g from the symbolic's per-level mapping);
// the lanes of a group split the node's destinations and its descendant
// list, and combine partial sums with a butterfly over the group.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "pf.h"
#include "pf_internal.h"
#include "pf_kernels.h"

using namespace pf;

// ===========================================================================
// device helpers
// ===========================================================================
namespace {

constexpr int kMaxThreads = 1024;

// Voltage accessors: stored rectangular voltages, or computed from polar.
struct EFArr {
    const double* e;
    const double* f;
    __device__ __forceinline__ void get(int k, double& ek, double& fk) const
    {
        ek = e[k];
        fk = f[k];
    }
};
struct EFPolar {
    const double* Vm;
    const double* Va;
    __device__ __forceinline__ void get(int k, double& ek, double& fk) const
    {
        double s, c;
        sincos(Va[k], &s, &c);
        ek = Vm[k] * c;
        fk = Vm[k] * s;
    }
};

// P_i + jQ_i = V_i conj(sum_k Y_ik V_k)  (nodal: one row of Y).
template <class EF>
__device__ __forceinline__ void injection(const DevSym& S, const double* __restrict__ yv,
                                          const EF& ef, int i, double& P, double& Q)
{
    double ir = 0.0, ii = 0.0;
    const int q1 = S.yptr[i + 1];
    for (int q = S.yptr[i]; q < q1; ++q) {
        const int k = S.ycol[q];
        const double2 y = reinterpret_cast<const double2*>(yv)[q];
        double ek, fk;
        ef.get(k, ek, fk);
        ir = fma(y.x, ek, fma(-y.y, fk, ir));
        ii = fma(y.x, fk, fma(y.y, ek, ii));
    }
    double ei, fi;
    ef.get(i, ei, fi);
    P = ei * ir + fi * ii;
    Q = fi * ir - ei * ii;
}

// Jacobian source reading the Newton state of one case.
template <class EF>
struct AsmState {
    const DevSym* S;
    const double* yv;
    const int8_t* type;
    const double* Vm;
    EF ef;
    const double* P;  // may be null: then computed on the fly
    const double* Q;

    __device__ __forceinline__ Blk diag(int j) const
    {
        const int bus = S->perm[j];
        const double2 y = reinterpret_cast<const double2*>(yv)[S->ydiag[j]];
        double p, q;
        if (P) {
            p = P[bus];
            q = Q[bus];
        } else {
            injection(*S, yv, ef, bus, p, q);
        }
        return jac_diag(y.x, y.y, p, q, Vm[bus], type[bus] == T_PV);
    }
    __device__ __forceinline__ void off(int j, int s, Blk& lo, Blk& up) const
    {
        const int ql = S->ylo[s];
        if (ql < 0) {  // fill-in: structurally present, numerically zero
            lo = bzero();
            up = bzero();
            return;
        }
        const int qu = S->yup[s];
        const int bj = S->perm[j], bk = S->perm[S->Li[s]];
        double ej, fj, ek, fk;
        ef.get(bj, ej, fj);
        ef.get(bk, ek, fk);
        const bool pj = type[bj] == T_PV, pk = type[bk] == T_PV;
        const double2 yl = reinterpret_cast<const double2*>(yv)[ql];
        const double2 yu = reinterpret_cast<const double2*>(yv)[qu];
        lo = jac_off(yl.x, yl.y, ek, fk, ej, fj, Vm[bj], pk, pj);  // block (k, j)
        up = jac_off(yu.x, yu.y, ej, fj, ek, fk, Vm[bk], pj, pk);  // block (j, k)
    }
};

// Jacobian source reading an assembled matrix in the filled layout.
struct AsmLoad {
    const double* D;
    const double* LU;
    __device__ __forceinline__ Blk diag(int j) const { return bload(D + 4 * (int64_t)j); }
    __device__ __forceinline__ void off(int, int s, Blk& lo, Blk& up) const
    {
        lo = bload(LU + 8 * (int64_t)s);
        up = bload(LU + 8 * (int64_t)s + 4);
    }
};

// Runs fn(node, lane, g) over the levels, up (1..p) or down (p..1), with a
// workgroup barrier after every level.
template <class F>
__device__ __forceinline__ void for_levels(const DevSym& S, bool up, F&& fn)
{
    for (int li = 0; li < S.nlev; ++li) {
        const int l = up ? li : S.nlev - 1 - li;
        const int g = S.level_g[l];
        const int beg = S.level_ptr[l];
        const int cnt = S.level_ptr[l + 1] - beg;
        const int gpb = blockDim.x / g;
        const int grp = threadIdx.x / g;
        const int lane = threadIdx.x & (g - 1);
        for (int base = 0; base < cnt; base += gpb) {
            const int idx = base + grp;
            if (idx < cnt) fn(S.level_nodes[beg + idx], lane, g);
        }
        __syncthreads();
    }
}

// Left-looking block LDU of node j (FactorizeGraphA, pull form).
//   D_j  = A_jj - sum_{i in R(j)} W_ji U_ij
//   W_kj = A_kj - sum_i W_ki U_ij,  V_jk = A_jk - sum_i W_ji U_ik  (k in S(j))
//   stored: D section <- D_j^-1, LU[s] <- (W_kj, U_jk = D_j^-1 V_jk)
// With FWD, also the forward substitution and normalisation of the rhs:
//   y_j = D_j^-1 (b_j - sum_{i in R(j)} W_ji y_i).
template <class ASM, bool FWD>
__device__ __forceinline__ void factor_node(const DevSym& S, const ASM& A, int j, int lane,
                                            int g, double* __restrict__ D,
                                            double* __restrict__ LU, double* __restrict__ rhs,
                                            int* s_bad)
{
    Blk ds = bzero();
    double z0 = 0.0, z1 = 0.0;
    const int r1 = S.Rp[j + 1];
    for (int r = S.Rp[j] + lane; r < r1; r += g) {
        const int b = S.Rs[r];
        const Blk w = bload(LU + 8 * (int64_t)b);
        const Blk u = bload(LU + 8 * (int64_t)b + 4);
        bmadd(ds, w, u);
        if (FWD) {
            const double2 yi = reinterpret_cast<const double2*>(rhs)[S.Ri[r]];
            mvadd(z0, z1, w, yi.x, yi.y);
        }
    }
    if (g > 1) {
        ds.a = gsum(ds.a, g);
        ds.b = gsum(ds.b, g);
        ds.c = gsum(ds.c, g);
        ds.d = gsum(ds.d, g);
        if (FWD) {
            z0 = gsum(z0, g);
            z1 = gsum(z1, g);
        }
    }
    const Blk Ajj = A.diag(j);
    const Blk Dj = {Ajj.a - ds.a, Ajj.b - ds.b, Ajj.c - ds.c, Ajj.d - ds.d};
    bool ok;
    const Blk Di = binv(Dj, ok);
    const int s1 = S.Lp[j + 1];
    for (int s = S.Lp[j] + lane; s < s1; s += g) {
        Blk Wk, Vk;
        A.off(j, s, Wk, Vk);
        const int u1 = S.Up[s + 1];
        for (int u = S.Up[s]; u < u1; ++u) {
            const int a = S.Ua[u], b = S.Ub[u];
            const Blk Wa = bload(LU + 8 * (int64_t)a);
            const Blk Uak = bload(LU + 8 * (int64_t)a + 4);
            const Blk Wb = bload(LU + 8 * (int64_t)b);
            const Blk Ubj = bload(LU + 8 * (int64_t)b + 4);
            bmsub(Wk, Wa, Ubj);
            bmsub(Vk, Wb, Uak);
        }
        bstore(LU + 8 * (int64_t)s, Wk);
        bstore(LU + 8 * (int64_t)s + 4, bmul(Di, Vk));
    }
    if (lane == 0) {
        if (!ok) *s_bad = 1;
        bstore(D + 4 * (int64_t)j, Di);
        if (FWD) {
            const double2 bj = reinterpret_cast<const double2*>(rhs)[j];
            const double x0 = bj.x - z0, x1 = bj.y - z1;
            double y0 = 0.0, y1 = 0.0;
            mvadd(y0, y1, Di, x0, x1);
            reinterpret_cast<double2*>(rhs)[j] = make_double2(y0, y1);
        }
    }
}

// Backward substitution of node j: x_j = y_j - sum_{k in S(j)} U_jk x_k.
// With the Newton update, also theta -= dtheta, |V| -= d|V| (PQ) and the
// rectangular voltage of the bus.
template <bool UPDATE>
__device__ __forceinline__ void back_node(const DevSym& S, int j, int lane, int g,
                                          const double* __restrict__ LU,
                                          double* __restrict__ rhs, const int8_t* type,
                                          double* Vm, double* Va, double* e, double* f)
{
    double a0 = 0.0, a1 = 0.0;
    const int s1 = S.Lp[j + 1];
    for (int s = S.Lp[j] + lane; s < s1; s += g) {
        const Blk u = bload(LU + 8 * (int64_t)s + 4);
        const double2 xk = reinterpret_cast<const double2*>(rhs)[S.Li[s]];
        mvadd(a0, a1, u, xk.x, xk.y);
    }
    if (g > 1) {
        a0 = gsum(a0, g);
        a1 = gsum(a1, g);
    }
    if (lane == 0) {
        const double2 y = reinterpret_cast<const double2*>(rhs)[j];
        const double x0 = y.x - a0, x1 = y.y - a1;
        reinterpret_cast<double2*>(rhs)[j] = make_double2(x0, x1);
        if (UPDATE) {
            const int bus = S.perm[j];
            const double va = Va[bus] - x0;
            double vm = Vm[bus];
            if (type[bus] != T_PV) vm -= x1;
            Va[bus] = va;
            Vm[bus] = vm;
            double sn, cs;
            sincos(va, &sn, &cs);
            e[bus] = vm * cs;
            f[bus] = vm * sn;
        }
    }
}

// Max over the workgroup with a NaN flag; every thread gets the result.
__device__ double block_max(double v, int nan, int& any_nan)
{
    __shared__ double s_v[kMaxThreads / 64 + 1];
    __shared__ int s_n[kMaxThreads / 64 + 1];
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    nan = __any(nan);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_v[w] = v;
        s_n[w] = nan;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        int fl = 0;
        for (int i = 0; i < (int)(blockDim.x + 63) / 64; ++i) {
            m = fmax(m, s_v[i]);
            fl |= s_n[i];
        }
        s_v[kMaxThreads / 64] = m;
        s_n[kMaxThreads / 64] = fl;
    }
    __syncthreads();
    const double r = s_v[kMaxThreads / 64];
    any_nan = s_n[kMaxThreads / 64];
    __syncthreads();
    return r;
}

// Mismatch of one case (all threads of the workgroup): P, Q per bus and the
// position-ordered rhs (F_P, F_Q), F_Q = 0 at PV buses.  Returns max |F|.
template <class EF>
__device__ double mismatch_case(const DevSym& S, const double* yv, const EF& ef,
                                const int8_t* type, const double* Psp, const double* Qsp,
                                double* P, double* Q, double* rhs, int& any_nan)
{
    double m = 0.0;
    int nan = 0;
    for (int i = threadIdx.x; i < S.n; i += blockDim.x) {
        double p, q;
        injection(S, yv, ef, i, p, q);
        if (P) {
            P[i] = p;
            Q[i] = q;
        }
        const int ps = S.pos[i];
        if (ps >= 0) {
            const double fp = p - Psp[i];
            const double fq = (type[i] == T_PV) ? 0.0 : q - Qsp[i];
            reinterpret_cast<double2*>(rhs)[ps] = make_double2(fp, fq);
            nan |= (fp != fp) | (fq != fq);
            m = fmax(m, fmax(fabs(fp), fabs(fq)));
        }
    }
    return block_max(m, nan, any_nan);
}

struct NewtonArgs {
    const double* yval;
    int64_t y_stride;
    const int8_t* type;
    int64_t type_stride;
    const double* Psp;
    const double* Qsp;
    int64_t inj_stride;
    double* Vm;
    double* Va;
    int64_t v_stride;
    double* ws;
    int64_t ws_stride;
    double tol;
    int max_iter;
    int flags;
    int32_t* iters;
    double* norm;
    int32_t* status;
};

struct CaseDesc {
    DevSym sym;
    int64_t bus_off, br_off, y_off, ws_off;
};

// The whole Newton-Raphson loop of one case, run by one workgroup.
__device__ void newton_case(const DevSym& S, const double* yv, const int8_t* type,
                            const double* Psp, const double* Qsp, double* Vm, double* Va,
                            double* ws, double tol, int max_iter, int flags, int32_t* o_iters,
                            double* o_norm, int32_t* o_status)
{
    __shared__ int s_bad;
    CaseState c = case_state(S, ws);
    for (int i = threadIdx.x; i < S.n; i += blockDim.x) {
        double sn, cs;
        sincos(Va[i], &sn, &cs);
        c.e[i] = Vm[i] * cs;
        c.f[i] = Vm[i] * sn;
    }
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    const EFArr ef{c.e, c.f};
    const AsmState<EFArr> A{&S, yv, type, Vm, ef, c.P, c.Q};
    int it = 0, st = ST_NOT_CONVERGED;
    double nrm = 0.0;
    for (;;) {
        int any_nan = 0;
        nrm = mismatch_case(S, yv, ef, type, Psp, Qsp, c.P, c.Q, c.rhs, any_nan);
        if (any_nan || !isfinite(nrm)) {
            st = ST_NONFINITE;
            break;
        }
        if (nrm < tol) {
            st = ST_OK;
            break;
        }
        if (it >= max_iter) {
            st = ST_NOT_CONVERGED;
            break;
        }
        for_levels(S, true, [&](int j, int lane, int g) {
            factor_node<AsmState<EFArr>, true>(S, A, j, lane, g, c.D, c.LU, c.rhs, &s_bad);
        });
        if (s_bad) {
            st = ST_ZERO_PIVOT;
            break;
        }
        for_levels(S, false, [&](int j, int lane, int g) {
            back_node<true>(S, j, lane, g, c.LU, c.rhs, type, Vm, Va, c.e, c.f);
        });
        ++it;
    }
    if ((flags & PF_NEWTON_KEEP_FACTORS) && st == ST_OK) {
        for_levels(S, true, [&](int j, int lane, int g) {
            factor_node<AsmState<EFArr>, false>(S, A, j, lane, g, c.D, c.LU, c.rhs, &s_bad);
        });
        if (s_bad) st = ST_ZERO_PIVOT;
    }
    if (threadIdx.x == 0) {
        if (o_iters) *o_iters = it;
        if (o_norm) *o_norm = nrm;
        if (o_status) *o_status = st;
    }
}

}  // namespace

// ===========================================================================
// kernels
// ===========================================================================
__global__ void k_ybus(DevSym S, const double* __restrict__ r, const double* __restrict__ x,
                       const double* __restrict__ bc, int64_t bstride,
                       double* __restrict__ yval, int64_t ystride)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= S.n) return;
    const double* rc = r + c * bstride;
    const double* xc = x + c * bstride;
    const double* bcc = bc + c * bstride;
    double* yc = yval + c * ystride;
    for (int q = S.yptr[i]; q < S.yptr[i + 1]; ++q) {
        const bool diag = S.ycol[q] == i;
        double G = 0.0, Bv = 0.0;
        for (int t = S.ybr_ptr[q]; t < S.ybr_ptr[q + 1]; ++t) {
            const int e = S.ybr[t];
            const double rr = rc[e], xx = xc[e];
            const double den = rr * rr + xx * xx;
            const double yg = rr / den, yb = -xx / den;
            if (diag) {
                G += yg;
                Bv += yb + 0.5 * bcc[e];
            } else {
                G -= yg;
                Bv -= yb;
            }
        }
        reinterpret_cast<double2*>(yc)[q] = make_double2(G, Bv);
    }
}

__global__ void k_ybus_multi(const CaseDesc* __restrict__ descs, const double* __restrict__ r,
                             const double* __restrict__ x, const double* __restrict__ bc,
                             double* __restrict__ yval)
{
    const CaseDesc& cd = descs[blockIdx.x];
    const DevSym& S = cd.sym;
    const double* rc = r + cd.br_off;
    const double* xc = x + cd.br_off;
    const double* bcc = bc + cd.br_off;
    double* yc = yval + cd.y_off;
    for (int i = threadIdx.x; i < S.n; i += blockDim.x) {
        for (int q = S.yptr[i]; q < S.yptr[i + 1]; ++q) {
            const bool diag = S.ycol[q] == i;
            double G = 0.0, Bv = 0.0;
            for (int t = S.ybr_ptr[q]; t < S.ybr_ptr[q + 1]; ++t) {
                const int e = S.ybr[t];
                const double rr = rc[e], xx = xc[e];
                const double den = rr * rr + xx * xx;
                const double yg = rr / den, yb = -xx / den;
                if (diag) {
                    G += yg;
                    Bv += yb + 0.5 * bcc[e];
                } else {
                    G -= yg;
                    Bv -= yb;
                }
            }
            reinterpret_cast<double2*>(yc)[q] = make_double2(G, Bv);
        }
    }
}

__global__ __launch_bounds__(kMaxThreads) void k_mismatch(
    DevSym S, const double* yval, int64_t y_stride, const int8_t* type, int64_t type_stride,
    const double* Psp, const double* Qsp, int64_t inj_stride, const double* Vm,
    const double* Va, int64_t v_stride, double* rhs, int64_t rhs_stride, double* norm,
    double* PQ)
{
    const int c = blockIdx.x;
    const EFPolar ef{Vm + c * v_stride, Va + c * v_stride};
    int any_nan = 0;
    double* pq = PQ ? PQ + (int64_t)c * 2 * S.n : nullptr;
    double m = 0.0;
    int nan = 0;
    const double* yv = yval + c * y_stride;
    const int8_t* ty = type + c * type_stride;
    const double* ps = Psp + c * inj_stride;
    const double* qs = Qsp + c * inj_stride;
    double* rh = rhs + c * rhs_stride;
    for (int i = threadIdx.x; i < S.n; i += blockDim.x) {
        double p, q;
        injection(S, yv, ef, i, p, q);
        if (pq) reinterpret_cast<double2*>(pq)[i] = make_double2(p, q);
        const int po = S.pos[i];
        if (po >= 0) {
            const double fp = p - ps[i];
            const double fq = (ty[i] == T_PV) ? 0.0 : q - qs[i];
            reinterpret_cast<double2*>(rh)[po] = make_double2(fp, fq);
            nan |= (fp != fp) | (fq != fq);
            m = fmax(m, fmax(fabs(fp), fabs(fq)));
        }
    }
    const double r = block_max(m, nan, any_nan);
    if (threadIdx.x == 0 && norm) norm[c] = any_nan ? __builtin_nan("") : r;
}

__global__ void k_jacobian(DevSym S, const double* yval, int64_t y_stride, const int8_t* type,
                           int64_t type_stride, const double* Vm, const double* Va,
                           int64_t v_stride, double* vals, int64_t vals_stride)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (j >= S.nn) return;
    const EFPolar ef{Vm + c * v_stride, Va + c * v_stride};
    const AsmState<EFPolar> A{&S, yval + c * y_stride, type + c * type_stride,
                              Vm + c * v_stride, ef, nullptr, nullptr};
    double* D = vals + c * vals_stride;
    double* LU = D + 4 * (int64_t)S.nn;
    bstore(D + 4 * (int64_t)j, A.diag(j));
    for (int s = S.Lp[j]; s < S.Lp[j + 1]; ++s) {
        Blk lo, up;
        A.off(j, s, lo, up);
        bstore(LU + 8 * (int64_t)s, lo);
        bstore(LU + 8 * (int64_t)s + 4, up);
    }
}

__global__ __launch_bounds__(kMaxThreads) void k_factor(DevSym S, double* vals,
                                                        int64_t vals_stride, int32_t* status)
{
    __shared__ int s_bad;
    const int c = blockIdx.x;
    double* D = vals + c * vals_stride;
    double* LU = D + 4 * (int64_t)S.nn;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    const AsmLoad A{D, LU};
    for_levels(S, true, [&](int j, int lane, int g) {
        factor_node<AsmLoad, false>(S, A, j, lane, g, D, LU, nullptr, &s_bad);
    });
    if (threadIdx.x == 0 && status) status[c] = s_bad ? ST_ZERO_PIVOT : ST_OK;
}

// transpose = 0: y_j = D_j^-1 (b_j - sum_{i in R(j)} W_ji y_i)  (levels up),
//                x_j = y_j - sum_{k in S(j)} U_jk x_k            (levels down).
// transpose = 1: p_j = g_j - sum_{i in R(j)} U_ij^T p_i           (levels up),
//                l_j = D_j^-T (p_j - sum_{k in S(j)} W_kj^T l_k)  (levels down).
template <bool TRANS>
__global__ __launch_bounds__(kMaxThreads) void k_solve(DevSym S, const double* vals,
                                                       int64_t vals_stride, double* rhs,
                                                       int64_t rhs_stride)
{
    const int c = blockIdx.x;
    const double* D = vals + c * vals_stride;
    const double* LU = D + 4 * (int64_t)S.nn;
    double* x = rhs + c * rhs_stride;
    double2* x2 = reinterpret_cast<double2*>(x);
    for_levels(S, true, [&](int j, int lane, int g) {
        double z0 = 0.0, z1 = 0.0;
        for (int r = S.Rp[j] + lane; r < S.Rp[j + 1]; r += g) {
            const double2 xi = x2[S.Ri[r]];
            const Blk M = bload(LU + 8 * (int64_t)S.Rs[r] + (TRANS ? 4 : 0));
            if (TRANS) mtvadd(z0, z1, M, xi.x, xi.y);
            else mvadd(z0, z1, M, xi.x, xi.y);
        }
        if (g > 1) {
            z0 = gsum(z0, g);
            z1 = gsum(z1, g);
        }
        if (lane == 0) {
            const double2 b = x2[j];
            double u0 = b.x - z0, u1 = b.y - z1;
            if (!TRANS) {
                const Blk Di = bload(D + 4 * (int64_t)j);
                double y0 = 0.0, y1 = 0.0;
                mvadd(y0, y1, Di, u0, u1);
                u0 = y0;
                u1 = y1;
            }
            x2[j] = make_double2(u0, u1);
        }
    });
    for_levels(S, false, [&](int j, int lane, int g) {
        double a0 = 0.0, a1 = 0.0;
        for (int s = S.Lp[j] + lane; s < S.Lp[j + 1]; s += g) {
            const double2 xk = x2[S.Li[s]];
            const Blk M = bload(LU + 8 * (int64_t)s + (TRANS ? 0 : 4));
            if (TRANS) mtvadd(a0, a1, M, xk.x, xk.y);
            else mvadd(a0, a1, M, xk.x, xk.y);
        }
        if (g > 1) {
            a0 = gsum(a0, g);
            a1 = gsum(a1, g);
        }
        if (lane == 0) {
            const double2 y = x2[j];
            double u0 = y.x - a0, u1 = y.y - a1;
            if (TRANS) {
                const Blk Di = bload(D + 4 * (int64_t)j);
                double l0 = 0.0, l1 = 0.0;
                mtvadd(l0, l1, Di, u0, u1);
                u0 = l0;
                u1 = l1;
            }
            x2[j] = make_double2(u0, u1);
        }
    });
}

template <bool MULTI>
__global__ __launch_bounds__(kMaxThreads) void k_newton(DevSym Sarg,
                                                        const CaseDesc* __restrict__ descs,
                                                        const int32_t* __restrict__ order,
                                                        NewtonArgs a)
{
    int c;
    if (MULTI) {
        c = order[blockIdx.x];
        const CaseDesc& cd = descs[c];
        const DevSym S = cd.sym;
        newton_case(S, a.yval + cd.y_off, a.type + cd.bus_off, a.Psp + cd.bus_off,
                    a.Qsp + cd.bus_off, a.Vm + cd.bus_off, a.Va + cd.bus_off,
                    a.ws + cd.ws_off, a.tol, a.max_iter, a.flags,
                    a.iters ? a.iters + c : nullptr, a.norm ? a.norm + c : nullptr,
                    a.status ? a.status + c : nullptr);
    } else {
        c = blockIdx.x;
        newton_case(Sarg, a.yval + c * a.y_stride, a.type + c * a.type_stride,
                    a.Psp + c * a.inj_stride, a.Qsp + c * a.inj_stride, a.Vm + c * a.v_stride,
                    a.Va + c * a.v_stride, a.ws + c * a.ws_stride, a.tol, a.max_iter,
                    a.flags, a.iters ? a.iters + c : nullptr, a.norm ? a.norm + c : nullptr,
                    a.status ? a.status + c : nullptr);
    }
}

__global__ void k_adj_rhs(DevSym S, const double* gVm, const double* gVa, int64_t v_stride,
                          const int8_t* type, int64_t type_stride, double* rhs,
                          int64_t rhs_stride)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (p >= S.nn) return;
    const int bus = S.perm[p];
    const double ga = gVa[c * v_stride + bus];
    const double gm = (type[c * type_stride + bus] == T_PV) ? 0.0 : gVm[c * v_stride + bus];
    reinterpret_cast<double2*>(rhs + c * rhs_stride)[p] = make_double2(ga, gm);
}

__global__ void k_adj_bus(DevSym S, const double* lam, int64_t lam_stride, const int8_t* type,
                          int64_t type_stride, double* gP, double* gQ, int64_t g_stride)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= S.n) return;
    const int p = S.pos[i];
    double lp = 0.0, lq = 0.0;
    if (p >= 0) {
        const double2 l = reinterpret_cast<const double2*>(lam + c * lam_stride)[p];
        lp = l.x;
        lq = (type[c * type_stride + i] == T_PV) ? 0.0 : l.y;
    }
    gP[c * g_stride + i] = lp;
    gQ[c * g_stride + i] = lq;
}

// dL/dx_e for one case: dS_f = V_f conj(dy (V_f - V_t)), dS_t = V_t conj(dy (V_t - V_f)),
// dy = -j y^2, gx = -(lamP_f Re dS_f + lamQ_f Im dS_f + same at t).
__device__ __forceinline__ double adj_branch(const DevSym& S, int e, int fb, int tb,
                                             const double* lam, const int8_t* type,
                                             const double* Vm, const double* Va, double r,
                                             double x)
{
    const double den = r * r + x * x;
    const double yr = r / den, yi = -x / den;
    const double dyr = 2.0 * yr * yi, dyi = -(yr * yr - yi * yi);
    double sf, cf, st, ct;
    sincos(Va[fb], &sf, &cf);
    sincos(Va[tb], &st, &ct);
    const double ef = Vm[fb] * cf, ff = Vm[fb] * sf;
    const double et = Vm[tb] * ct, ft = Vm[tb] * st;
    const double dr = ef - et, di = ff - ft;
    const double cr = dyr * dr - dyi * di, ci = dyr * di + dyi * dr;
    double acc = 0.0;
    const int pf_ = S.pos[fb], pt_ = S.pos[tb];
    const double2* l2 = reinterpret_cast<const double2*>(lam);
    if (pf_ >= 0) {
        const double2 l = l2[pf_];
        const double lq = (type[fb] == T_PV) ? 0.0 : l.y;
        acc += l.x * (ef * cr + ff * ci) + lq * (ff * cr - ef * ci);
    }
    if (pt_ >= 0) {
        const double2 l = l2[pt_];
        const double lq = (type[tb] == T_PV) ? 0.0 : l.y;
        acc += l.x * (-(et * cr + ft * ci)) + lq * (-(ft * cr - et * ci));
    }
    (void)e;
    return -acc;
}

__global__ void k_adj_branch(DevSym S, const int32_t* __restrict__ from,
                             const int32_t* __restrict__ to, int B, const double* lam,
                             int64_t lam_stride, const int8_t* type, int64_t type_stride,
                             const double* Vm, const double* Va, int64_t v_stride,
                             const double* r, const double* x, int64_t branch_stride,
                             double* gx, int mode)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= S.m) return;
    const int fb = from[e], tb = to[e];
    if (mode == 1) {
        double acc = 0.0;
        for (int c = 0; c < B; ++c)
            acc += adj_branch(S, e, fb, tb, lam + c * lam_stride, type + c * type_stride,
                              Vm + c * v_stride, Va + c * v_stride, r[c * branch_stride + e],
                              x[c * branch_stride + e]);
        gx[e] = acc;
    } else {
        const int c = blockIdx.y;
        gx[(int64_t)c * S.m + e] =
            adj_branch(S, e, fb, tb, lam + c * lam_stride, type + c * type_stride,
                       Vm + c * v_stride, Va + c * v_stride, r[c * branch_stride + e],
                       x[c * branch_stride + e]);
    }
}

// ===========================================================================
// C ABI
// ===========================================================================
struct pf_symbolic_s {
    HostSym h;
    int threads = 256;
    const int32_t* d_from = nullptr;  // device copies of the branch ends
    const int32_t* d_to = nullptr;
};

struct pf_multi_s {
    std::vector<pf_symbolic> syms;
    std::vector<int64_t> bus_off, br_off, y_off, ws_off;
    std::vector<int32_t> order;
    int threads = 256;
    const CaseDesc* d_desc = nullptr;
    const int32_t* d_order = nullptr;
    bool uploaded = false;
};

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

int hip_check(hipError_t e, const char* what)
{
    if (e != hipSuccess)
        return fail(PF_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
    return PF_OK;
}

int launch_check(const char* what) { return hip_check(hipGetLastError(), what); }

bool ready(const pf_symbolic s, const char* fn)
{
    if (!s) {
        fail(PF_E_INVALID, std::string(fn) + ": NULL symbolic");
        return false;
    }
    if (!s->h.uploaded) {
        fail(PF_E_INVALID, std::string(fn) + ": symbolic not uploaded");
        return false;
    }
    return true;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace

extern "C" {

const char* pf_version(void) { return "libpf 0.1 gfx950"; }

const char* pf_status_string(int st)
{
    switch (st) {
        case PF_OK: return "ok";
        case PF_E_INVALID: return "invalid argument";
        case PF_E_HIP: return "HIP runtime error";
        case PF_E_WORKSPACE: return "workspace too small";
        case PF_E_DISCONNECTED: return "grid not connected to the slack";
        case PF_E_ZERO_PIVOT: return "zero pivot";
        case PF_E_NOT_CONVERGED: return "not converged";
        case PF_E_NONFINITE: return "non-finite mismatch";
        default: return "unknown status";
    }
}

const char* pf_last_error(void) { return g_err.c_str(); }

int pf_analyze(int n, int m, const int32_t* from, const int32_t* to, int slack, int ordering,
               pf_symbolic* out)
{
    if (!out) return fail(PF_E_INVALID, "pf_analyze: out is NULL");
    *out = nullptr;
    try {
        pf_symbolic s = new pf_symbolic_s();
        std::string msg;
        int rc = pf::analyze(n, m, from, to, slack, ordering, s->h, msg);
        if (rc != PF_OK) {
            delete s;
            return fail(rc, msg);
        }
        *out = s;
        g_err.clear();
        return PF_OK;
    } catch (const std::exception& ex) {
        return fail(PF_E_INVALID, std::string("pf_analyze: ") + ex.what());
    }
}

int pf_symbolic_info(const pf_symbolic s, pf_info* info)
{
    if (!s || !info) return fail(PF_E_INVALID, "pf_symbolic_info: NULL argument");
    const HostSym& h = s->h;
    info->n = h.n;
    info->m = h.m;
    info->nn = h.nn;
    info->slack = h.slack;
    info->nnz_y = (int64_t)h.ycol.size();
    info->nnz_l = (int64_t)h.Li.size();
    info->n_upd = (int64_t)h.Ua.size();
    info->nlevels = (int32_t)h.level_ptr.size() - 1;
    info->max_level_width = h.max_width;
    info->vals_doubles = h.vals_doubles();
    info->ws_doubles = h.ws_doubles();
    info->dev_bytes = h.dev_bytes() + 2 * ((std::max<size_t>(h.m, 1) * 4 + 255) & ~(size_t)255);
    return PF_OK;
}

int pf_symbolic_export(const pf_symbolic s, int32_t* perm, int32_t* parent, int32_t* level,
                       int32_t* level_ptr, int32_t* level_nodes, int32_t* Lp, int32_t* Li)
{
    if (!s) return fail(PF_E_INVALID, "pf_symbolic_export: NULL symbolic");
    const HostSym& h = s->h;
    auto cp = [](int32_t* dst, const std::vector<int32_t>& v) {
        if (dst && !v.empty()) std::memcpy(dst, v.data(), v.size() * sizeof(int32_t));
    };
    cp(perm, h.perm);
    cp(parent, h.parent);
    cp(level, h.level);
    cp(level_ptr, h.level_ptr);
    cp(level_nodes, h.level_nodes);
    cp(Lp, h.Lp);
    cp(Li, h.Li);
    return PF_OK;
}

int pf_symbolic_ybus_pattern(const pf_symbolic s, int32_t* yptr, int32_t* ycol)
{
    if (!s) return fail(PF_E_INVALID, "pf_symbolic_ybus_pattern: NULL symbolic");
    if (yptr) std::memcpy(yptr, s->h.yptr.data(), s->h.yptr.size() * sizeof(int32_t));
    if (ycol && !s->h.ycol.empty())
        std::memcpy(ycol, s->h.ycol.data(), s->h.ycol.size() * sizeof(int32_t));
    return PF_OK;
}

int pf_symbolic_set_mapping(pf_symbolic s, const int32_t* lanes)
{
    if (!s || !lanes) return fail(PF_E_INVALID, "pf_symbolic_set_mapping: NULL argument");
    int nlev = (int)s->h.level_ptr.size() - 1;
    for (int l = 0; l < nlev; ++l) {
        int g = lanes[l];
        if (g < 1 || g > 64 || (g & (g - 1)))
            return fail(PF_E_INVALID, "pf_symbolic_set_mapping: lanes must be 1,2,4,...,64");
    }
    for (int l = 0; l < nlev; ++l) s->h.level_g[l] = lanes[l];
    return PF_OK;
}

int pf_symbolic_get_mapping(const pf_symbolic s, int32_t* lanes)
{
    if (!s || !lanes) return fail(PF_E_INVALID, "pf_symbolic_get_mapping: NULL argument");
    int nlev = (int)s->h.level_ptr.size() - 1;
    for (int l = 0; l < nlev; ++l) lanes[l] = s->h.level_g[l];
    return PF_OK;
}

int pf_symbolic_upload(pf_symbolic s, void* d_buf, size_t bytes, void* stream)
{
    if (!s || !d_buf) return fail(PF_E_INVALID, "pf_symbolic_upload: NULL argument");
    HostSym& h = s->h;
    pf_info info;
    pf_symbolic_info(s, &info);
    if (bytes < info.dev_bytes)
        return fail(PF_E_WORKSPACE, "pf_symbolic_upload: buffer smaller than info.dev_bytes");
    if (reinterpret_cast<uintptr_t>(d_buf) & 255)
        return fail(PF_E_WORKSPACE, "pf_symbolic_upload: buffer not 256-byte aligned");
    std::vector<char> stage(info.dev_bytes, 0);
    char* base = static_cast<char*>(d_buf);
    size_t off = 0;
    auto put = [&](const std::vector<int32_t>& v) -> const int32_t* {
        size_t nb = std::max<size_t>(v.size(), 1) * sizeof(int32_t);
        if (!v.empty()) std::memcpy(stage.data() + off, v.data(), v.size() * sizeof(int32_t));
        const int32_t* dptr = reinterpret_cast<const int32_t*>(base + off);
        off += (nb + 255) & ~(size_t)255;
        return dptr;
    };
    DevSym d{};
    d.n = h.n;
    d.m = h.m;
    d.nn = h.nn;
    d.slack = h.slack;
    d.nnz_y = (int32_t)h.ycol.size();
    d.nnz_l = (int32_t)h.Li.size();
    d.nlev = (int32_t)h.level_ptr.size() - 1;
    d.n_upd = (int64_t)h.Ua.size();
    d.vals_doubles = h.vals_doubles();
    d.ws_doubles = h.ws_doubles();
    d.yptr = put(h.yptr);
    d.ycol = put(h.ycol);
    d.ybr_ptr = put(h.ybr_ptr);
    d.ybr = put(h.ybr);
    d.perm = put(h.perm);
    d.pos = put(h.pos);
    d.Lp = put(h.Lp);
    d.Li = put(h.Li);
    d.ylo = put(h.ylo);
    d.yup = put(h.yup);
    d.ydiag = put(h.ydiag);
    d.Rp = put(h.Rp);
    d.Ri = put(h.Ri);
    d.Rs = put(h.Rs);
    d.Up = put(h.Up);
    d.Ua = put(h.Ua);
    d.Ub = put(h.Ub);
    d.level_ptr = put(h.level_ptr);
    d.level_nodes = put(h.level_nodes);
    d.level_g = put(h.level_g);
    s->d_from = put(h.from);
    s->d_to = put(h.to);
    if (off > info.dev_bytes) return fail(PF_E_WORKSPACE, "pf_symbolic_upload: size mismatch");
    int rc = hip_check(hipMemcpyAsync(d_buf, stage.data(), off, hipMemcpyHostToDevice,
                                      as_stream(stream)),
                       "pf_symbolic_upload: hipMemcpyAsync");
    if (rc) return rc;
    rc = hip_check(hipStreamSynchronize(as_stream(stream)), "pf_symbolic_upload: sync");
    if (rc) return rc;
    h.dev = d;
    h.uploaded = true;
    return PF_OK;
}

void pf_symbolic_destroy(pf_symbolic s) { delete s; }

int pf_build_ybus(const pf_symbolic s, int B, const double* d_r, const double* d_x,
                  const double* d_b, int64_t branch_stride, double* d_yval, int64_t y_stride,
                  void* stream)
{
    if (!ready(s, "pf_build_ybus")) return PF_E_INVALID;
    if (B < 0 || B > 65535 || !d_r || !d_x || !d_b || !d_yval)
        return fail(PF_E_INVALID, "pf_build_ybus: bad arguments");
    if (B > 1 && y_stride < 2 * (int64_t)s->h.ycol.size())
        return fail(PF_E_WORKSPACE, "pf_build_ybus: y_stride < 2*nnz_y");
    if (B == 0) return PF_OK;
    dim3 grid((s->h.n + 255) / 256, B);
    hipLaunchKernelGGL(k_ybus, grid, dim3(256), 0, as_stream(stream), s->h.dev, d_r, d_x, d_b,
                       branch_stride, d_yval, y_stride);
    return launch_check("pf_build_ybus");
}

int pf_mismatch(const pf_symbolic s, int B, const double* d_yval, int64_t y_stride,
                const int8_t* d_type, int64_t type_stride, const double* d_Psp,
                const double* d_Qsp, int64_t inj_stride, const double* d_Vm, const double* d_Va,
                int64_t v_stride, double* d_rhs, int64_t rhs_stride, double* d_norm,
                double* d_PQ, void* stream)
{
    if (!ready(s, "pf_mismatch")) return PF_E_INVALID;
    if (B < 0 || !d_yval || !d_type || !d_Psp || !d_Qsp || !d_Vm || !d_Va || !d_rhs)
        return fail(PF_E_INVALID, "pf_mismatch: bad arguments");
    if (B == 0) return PF_OK;
    hipLaunchKernelGGL(k_mismatch, dim3(B), dim3(256), 0, as_stream(stream), s->h.dev, d_yval,
                       y_stride, d_type, type_stride, d_Psp, d_Qsp, inj_stride, d_Vm, d_Va,
                       v_stride, d_rhs, rhs_stride, d_norm, d_PQ);
    return launch_check("pf_mismatch");
}

int pf_jacobian(const pf_symbolic s, int B, const double* d_yval, int64_t y_stride,
                const int8_t* d_type, int64_t type_stride, const double* d_Vm, const double* d_Va,
                int64_t v_stride, double* d_vals, int64_t vals_stride, void* stream)
{
    if (!ready(s, "pf_jacobian")) return PF_E_INVALID;
    if (B < 0 || B > 65535 || !d_yval || !d_type || !d_Vm || !d_Va || !d_vals)
        return fail(PF_E_INVALID, "pf_jacobian: bad arguments");
    if (B > 1 && vals_stride < s->h.vals_doubles())
        return fail(PF_E_WORKSPACE, "pf_jacobian: vals_stride < vals_doubles");
    if (B == 0 || s->h.nn == 0) return PF_OK;
    dim3 grid((s->h.nn + 255) / 256, B);
    hipLaunchKernelGGL(k_jacobian, grid, dim3(256), 0, as_stream(stream), s->h.dev, d_yval,
                       y_stride, d_type, type_stride, d_Vm, d_Va, v_stride, d_vals, vals_stride);
    return launch_check("pf_jacobian");
}

int pf_factor(const pf_symbolic s, int B, double* d_vals, int64_t vals_stride,
              int32_t* d_status, void* stream)
{
    if (!ready(s, "pf_factor")) return PF_E_INVALID;
    if (B < 0 || !d_vals) return fail(PF_E_INVALID, "pf_factor: bad arguments");
    if (B > 1 && vals_stride < s->h.vals_doubles())
        return fail(PF_E_WORKSPACE, "pf_factor: vals_stride < vals_doubles");
    if (B == 0) return PF_OK;
    hipLaunchKernelGGL(k_factor, dim3(B), dim3(s->threads), 0, as_stream(stream), s->h.dev,
                       d_vals, vals_stride, d_status);
    return launch_check("pf_factor");
}

int pf_solve(const pf_symbolic s, int B, const double* d_vals, int64_t vals_stride,
             double* d_rhs, int64_t rhs_stride, int transpose, void* stream)
{
    if (!ready(s, "pf_solve")) return PF_E_INVALID;
    if (B < 0 || !d_vals || !d_rhs || (transpose != 0 && transpose != 1))
        return fail(PF_E_INVALID, "pf_solve: bad arguments");
    if (B > 1 && rhs_stride < 2 * (int64_t)s->h.nn)
        return fail(PF_E_WORKSPACE, "pf_solve: rhs_stride < 2*nn");
    if (B == 0) return PF_OK;
    if (transpose)
        hipLaunchKernelGGL(k_solve<true>, dim3(B), dim3(s->threads), 0, as_stream(stream),
                           s->h.dev, d_vals, vals_stride, d_rhs, rhs_stride);
    else
        hipLaunchKernelGGL(k_solve<false>, dim3(B), dim3(s->threads), 0, as_stream(stream),
                           s->h.dev, d_vals, vals_stride, d_rhs, rhs_stride);
    return launch_check("pf_solve");
}

int pf_newton(const pf_symbolic s, int B, const double* d_yval, int64_t y_stride,
              const int8_t* d_type, int64_t type_stride, const double* d_Psp,
              const double* d_Qsp, int64_t inj_stride, double* d_Vm, double* d_Va,
              int64_t v_stride, double tol, int max_iter, int flags, double* d_ws,
              int64_t ws_stride, int32_t* d_iters, double* d_norm, int32_t* d_status,
              void* stream)
{
    if (!ready(s, "pf_newton")) return PF_E_INVALID;
    if (B < 0 || max_iter < 0 || !(tol >= 0.0) || !d_yval || !d_type || !d_Psp || !d_Qsp ||
        !d_Vm || !d_Va || !d_ws)
        return fail(PF_E_INVALID, "pf_newton: bad arguments");
    if (B > 1 && (ws_stride < s->h.ws_doubles() || v_stride < s->h.n))
        return fail(PF_E_WORKSPACE, "pf_newton: ws_stride or v_stride too small");
    if (reinterpret_cast<uintptr_t>(d_ws) & 15)
        return fail(PF_E_WORKSPACE, "pf_newton: workspace must be 16-byte aligned");
    if (B == 0) return PF_OK;
    NewtonArgs a{d_yval, y_stride, d_type, type_stride, d_Psp, d_Qsp, inj_stride, d_Vm, d_Va,
                 v_stride, d_ws, ws_stride, tol, max_iter, flags, d_iters, d_norm, d_status};
    hipLaunchKernelGGL(k_newton<false>, dim3(B), dim3(s->threads), 0, as_stream(stream),
                       s->h.dev, (const CaseDesc*)nullptr, (const int32_t*)nullptr, a);
    return launch_check("pf_newton");
}

int pf_adjoint_params(const pf_symbolic s, int B, const double* d_lam, int64_t lam_stride,
                      const int8_t* d_type, int64_t type_stride, const double* d_Vm,
                      const double* d_Va, int64_t v_stride, const double* d_r,
                      const double* d_x, int64_t branch_stride, double* d_gP, double* d_gQ,
                      int64_t g_stride, double* d_gx, int gx_mode, void* stream)
{
    if (!ready(s, "pf_adjoint_params")) return PF_E_INVALID;
    if (B < 0 || B > 65535 || !d_lam || !d_type || !d_Vm || !d_Va ||
        (gx_mode != 0 && gx_mode != 1))
        return fail(PF_E_INVALID, "pf_adjoint_params: bad arguments");
    if (B == 0) return PF_OK;
    if (d_gP && d_gQ) {
        dim3 grid((s->h.n + 255) / 256, B);
        hipLaunchKernelGGL(k_adj_bus, grid, dim3(256), 0, as_stream(stream), s->h.dev, d_lam,
                           lam_stride, d_type, type_stride, d_gP, d_gQ, g_stride);
        int rc = launch_check("pf_adjoint_params");
        if (rc) return rc;
    }
    if (d_gx && s->h.m > 0) {
        if (!d_r || !d_x) return fail(PF_E_INVALID, "pf_adjoint_params: need r and x");
        dim3 grid((s->h.m + 255) / 256, gx_mode == 1 ? 1 : B);
        hipLaunchKernelGGL(k_adj_branch, grid, dim3(256), 0, as_stream(stream), s->h.dev,
                           s->d_from, s->d_to, B, d_lam, lam_stride, d_type, type_stride, d_Vm,
                           d_Va, v_stride, d_r, d_x, branch_stride, d_gx, gx_mode);
        return launch_check("pf_adjoint_params");
    }
    return PF_OK;
}

int pf_adjoint_rhs(const pf_symbolic s, int B, const double* d_gVm, const double* d_gVa,
                   int64_t v_stride, const int8_t* d_type, int64_t type_stride, double* d_rhs,
                   int64_t rhs_stride, void* stream)
{
    if (!ready(s, "pf_adjoint_rhs")) return PF_E_INVALID;
    if (B < 0 || B > 65535 || !d_gVm || !d_gVa || !d_type || !d_rhs)
        return fail(PF_E_INVALID, "pf_adjoint_rhs: bad arguments");
    if (B > 1 && rhs_stride < 2 * (int64_t)s->h.nn)
        return fail(PF_E_WORKSPACE, "pf_adjoint_rhs: rhs_stride < 2*nn");
    if (B == 0) return PF_OK;
    dim3 grid((s->h.nn + 255) / 256, B);
    hipLaunchKernelGGL(k_adj_rhs, grid, dim3(256), 0, as_stream(stream), s->h.dev, d_gVm,
                       d_gVa, v_stride, d_type, type_stride, d_rhs, rhs_stride);
    return launch_check("pf_adjoint_rhs");
}

// ---- multi-pattern batches -----------------------------------------------
int pf_multi_create(int G, const pf_symbolic* syms, pf_multi* out)
{
    if (!out || G < 0 || (G > 0 && !syms)) return fail(PF_E_INVALID, "pf_multi_create: bad args");
    *out = nullptr;
    pf_multi p = new pf_multi_s();
    p->syms.assign(syms, syms + G);
    p->bus_off.assign(G + 1, 0);
    p->br_off.assign(G + 1, 0);
    p->y_off.assign(G + 1, 0);
    p->ws_off.assign(G + 1, 0);
    std::vector<int64_t> work(G);
    for (int g = 0; g < G; ++g) {
        if (!syms[g]) {
            delete p;
            return fail(PF_E_INVALID, "pf_multi_create: NULL symbolic");
        }
        const HostSym& h = syms[g]->h;
        p->bus_off[g + 1] = p->bus_off[g] + h.n;
        p->br_off[g + 1] = p->br_off[g] + h.m;
        p->y_off[g + 1] = p->y_off[g] + 2 * (int64_t)h.ycol.size();
        p->ws_off[g + 1] = p->ws_off[g] + h.ws_doubles();
        work[g] = (int64_t)h.Ua.size() + 4 * (int64_t)h.Li.size() + 8 * (int64_t)h.n +
                  64 * (int64_t)(h.level_ptr.size());
    }
    p->order.resize(G);
    std::iota(p->order.begin(), p->order.end(), 0);
    std::stable_sort(p->order.begin(), p->order.end(),
                     [&](int a, int b) { return work[a] > work[b]; });
    *out = p;
    return PF_OK;
}

int pf_multi_info(const pf_multi p, size_t* dev_bytes, int64_t* bus_off, int64_t* branch_off,
                  int64_t* y_off, int64_t* ws_off)
{
    if (!p) return fail(PF_E_INVALID, "pf_multi_info: NULL plan");
    size_t G = p->syms.size();
    if (dev_bytes)
        *dev_bytes = ((G * sizeof(CaseDesc) + 255) & ~(size_t)255) +
                     ((std::max<size_t>(G, 1) * 4 + 255) & ~(size_t)255);
    auto cp = [&](int64_t* dst, const std::vector<int64_t>& v) {
        if (dst) std::memcpy(dst, v.data(), v.size() * sizeof(int64_t));
    };
    cp(bus_off, p->bus_off);
    cp(branch_off, p->br_off);
    cp(y_off, p->y_off);
    cp(ws_off, p->ws_off);
    return PF_OK;
}

int pf_multi_upload(pf_multi p, void* d_buf, size_t bytes, void* stream)
{
    if (!p || !d_buf) return fail(PF_E_INVALID, "pf_multi_upload: NULL argument");
    size_t need;
    pf_multi_info(p, &need, nullptr, nullptr, nullptr, nullptr);
    if (bytes < need) return fail(PF_E_WORKSPACE, "pf_multi_upload: buffer too small");
    if (reinterpret_cast<uintptr_t>(d_buf) & 255)
        return fail(PF_E_WORKSPACE, "pf_multi_upload: buffer not 256-byte aligned");
    size_t G = p->syms.size();
    std::vector<char> stage(need, 0);
    CaseDesc* cd = reinterpret_cast<CaseDesc*>(stage.data());
    for (size_t g = 0; g < G; ++g) {
        if (!p->syms[g]->h.uploaded)
            return fail(PF_E_INVALID, "pf_multi_upload: a symbolic is not uploaded");
        cd[g].sym = p->syms[g]->h.dev;
        cd[g].bus_off = p->bus_off[g];
        cd[g].br_off = p->br_off[g];
        cd[g].y_off = p->y_off[g];
        cd[g].ws_off = p->ws_off[g];
    }
    size_t ooff = (G * sizeof(CaseDesc) + 255) & ~(size_t)255;
    if (G) std::memcpy(stage.data() + ooff, p->order.data(), G * sizeof(int32_t));
    int rc = hip_check(hipMemcpyAsync(d_buf, stage.data(), need, hipMemcpyHostToDevice,
                                      as_stream(stream)),
                       "pf_multi_upload: hipMemcpyAsync");
    if (rc) return rc;
    rc = hip_check(hipStreamSynchronize(as_stream(stream)), "pf_multi_upload: sync");
    if (rc) return rc;
    p->d_desc = reinterpret_cast<const CaseDesc*>(d_buf);
    p->d_order = reinterpret_cast<const int32_t*>(static_cast<char*>(d_buf) + ooff);
    p->uploaded = true;
    return PF_OK;
}

int pf_build_ybus_multi(const pf_multi p, const double* d_r, const double* d_x,
                        const double* d_b, double* d_yval, void* stream)
{
    if (!p || !p->uploaded) return fail(PF_E_INVALID, "pf_build_ybus_multi: plan not uploaded");
    if (!d_r || !d_x || !d_b || !d_yval) return fail(PF_E_INVALID, "pf_build_ybus_multi: NULL");
    if (p->syms.empty()) return PF_OK;
    hipLaunchKernelGGL(k_ybus_multi, dim3(p->syms.size()), dim3(256), 0, as_stream(stream),
                       p->d_desc, d_r, d_x, d_b, d_yval);
    return launch_check("pf_build_ybus_multi");
}

int pf_newton_multi(const pf_multi p, const double* d_yval, const int8_t* d_type,
                    const double* d_Psp, const double* d_Qsp, double* d_Vm, double* d_Va,
                    double tol, int max_iter, int flags, double* d_ws, int32_t* d_iters,
                    double* d_norm, int32_t* d_status, void* stream)
{
    if (!p || !p->uploaded) return fail(PF_E_INVALID, "pf_newton_multi: plan not uploaded");
    if (max_iter < 0 || !(tol >= 0.0) || !d_yval || !d_type || !d_Psp || !d_Qsp || !d_Vm ||
        !d_Va || !d_ws)
        return fail(PF_E_INVALID, "pf_newton_multi: bad arguments");
    if (reinterpret_cast<uintptr_t>(d_ws) & 15)
        return fail(PF_E_WORKSPACE, "pf_newton_multi: workspace must be 16-byte aligned");
    if (p->syms.empty()) return PF_OK;
    NewtonArgs a{d_yval, 0, d_type, 0, d_Psp, d_Qsp, 0, d_Vm, d_Va, 0, d_ws, 0, tol, max_iter,
                 flags, d_iters, d_norm, d_status};
    DevSym none{};
    hipLaunchKernelGGL(k_newton<true>, dim3(p->syms.size()), dim3(p->threads), 0,
                       as_stream(stream), none, p->d_desc, p->d_order, a);
    return launch_check("pf_newton_multi");
}

void pf_multi_destroy(pf_multi p) { delete p; }

}  // extern "C"
