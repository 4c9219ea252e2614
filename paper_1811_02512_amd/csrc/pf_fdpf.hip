// libpf fast decoupled power flow and branch flows (device code, kernels and
// their C ABI entry points).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <numeric>
#include <string>
#include <type_traits>
#include <vector>

#include "pf.h"
#include "pf_device.h"
#include "pf_host.h"

using namespace pf::abi;

namespace {

// ---------------------------------------------------------------------------
// Fast decoupled power flow (Sec. III names it beside NR; Table III times it),
// XB matrices: B' from branch reactances only, B'' = -Im(Y) of the full
// pi-model, both symmetric, so the paper's factorisation is LDL^T (eqs. 1-3)
// with scalar elements.  Per matrix: d section [fd_lu] then (w, u) per slot
// with w_kj = l_kj d_j and u_jk = l_kj; after factorisation d holds 1/d_j.
// B'' of a PV bus is the identity row and column, so its |V| never moves.
// ---------------------------------------------------------------------------

// Entry of B' (XB = false) or B'' from the branches of admittance entry q.
template <bool XB>
__device__ __forceinline__ double fd_entry(const DevSym& S, int q, bool diag,
                                           const double* __restrict__ r,
                                           const double* __restrict__ x,
                                           const double* __restrict__ b)
{
    double v = 0.0;
    for (int t = S.ybr_ptr[q]; t < S.ybr_ptr[q + 1]; ++t) {
        const int e = S.ybr[t];
        if (!XB) {
            const double bx = 1.0 / x[e];
            v += diag ? bx : -bx;
        } else {
            const double rr = r[e], xx = x[e];
            const double bs = xx / (rr * rr + xx * xx);
            v += diag ? bs - b[e] / 2.0 : -bs;
        }
    }
    return v;
}

// Left-looking LDL^T of one node (pull form, like factor_node with 1x1
// blocks and U = L^T):
//   d_j = a_jj - sum_{i in R(j)} w_ji u_ij,
//   w_kj = a_kj - sum_i w_ki u_ij (k in S(j)),  u_jk = w_kj / d_j.
__device__ __forceinline__ void fd_factor_node(const DevSym& S, const NodeRec& rec, int lane,
                                               int g, double* m, int* s_bad)
{
    const int j = rec.a.x;
    double2* sl = reinterpret_cast<double2*>(m + S.fd_lu);
    double ds = 0.0;
    for (int r = rec.a.z + lane; r < rec.a.w; r += g) {
        const double2 wu = sl[S.rl[r].y];
        ds = fma(wu.x, wu.y, ds);
    }
    if (g > 1) ds = gsum(ds, g);
    const double D = m[j] - ds;
    const bool ok = D != 0.0 && isfinite(D);
    const double Dinv = 1.0 / D;
    for (int s = rec.b.x + lane; s < rec.b.y; s += g) {
        const int4 b = S.slot_info[2 * s + 1];
        double W = sl[s].x;
        for (int u = b.x; u < b.y; ++u) {
            const int2 p = S.upd[u];
            W = fma(-sl[p.x].x, sl[p.y].y, W);
        }
        sl[s] = make_double2(W, W * Dinv);
    }
    if (lane == 0) {
        m[j] = Dinv;
        if (!ok) *s_bad = 1;
    }
}

// Forward substitution and normalisation on component comp of the rhs:
//   y_j = (1/d_j) (b_j - sum_{i in R(j)} w_ji y_i), levels [0, l1) upward.
// Four entries per lane per batch with the next batch's indices in flight;
// the node's own b_j and 1/d_j are requested first.
// The work vector of a half step: with VL in LDS by position (xv), else the
// rhs component comp in the bus view.  The right-hand side b itself always
// comes from the rhs (the mismatch pass writes it there).
template <bool VL>
__device__ __forceinline__ double& fd_x(double* xv, const View& wb, int64_t rhs, int comp, int p)
{
    return VL ? xv[p] : *wb.at(rhs + 2 * (int64_t)p + comp);
}

template <bool VL>
__device__ __forceinline__ void fd_forward(const DevSym& S, const double* m, const View& wb,
                                           int64_t rhs, int comp, int l1, double* xv)
{
    const double2* sl = reinterpret_cast<const double2*>(m + S.fd_lu);
    for_nodes(S, 0, l1, true, [&](int, const NodeRec& rec, int lane, int g) {
        const int j = rec.a.x, r1 = rec.a.w;
        const double bj = *wb.at(rhs + 2 * (int64_t)j + comp);
        const double dj = m[j];
        int r = rec.a.z + lane;
        // absent entries are not loaded (skipped when no lane needs them)
        int2 e[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            e[k] = make_int2(0, 0);
            if (r + k * g < r1) e[k] = S.rl[r + k * g];
        }
        double z = 0.0;
        for (; r < r1; r += 4 * g) {
            double w[4], y[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                w[k] = 0.0;
                y[k] = 0.0;
                if (r + k * g < r1) {
                    w[k] = sl[e[k].y].x;
                    y[k] = fd_x<VL>(xv, wb, rhs, comp, e[k].x);
                }
            }
            const int rn = r + 4 * g;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (rn + k * g < r1) e[k] = S.rl[rn + k * g];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (r + k * g < r1) z = fma(w[k], y[k], z);
        }
        if (g > 1) z = gsum(z, g);
        if (lane == 0) fd_x<VL>(xv, wb, rhs, comp, j) = dj * (bj - z);
    });
}

// The half step at a bus: ANGLE: theta -= x; else |V| -= x at PQ buses.
template <bool ANGLE>
__device__ __forceinline__ void fd_half_step_to(const View& wb, int64_t br, const Blk& v, int bus,
                                                const PvMask& pv, double x)
{
    double vm = v.c, va = v.d;
    if (ANGLE) va -= x;
    else if (!pv(bus)) vm -= x;
    double sn, cs;
    sincos(va, &sn, &cs);
    wb.put(br, {vm * cs, vm * sn, vm, va});
}

template <bool ANGLE>
__device__ __forceinline__ void fd_half_step(const View& wb, int64_t bus_off, int bus,
                                             const PvMask& pv, double x)
{
    const int64_t br = bus_off + 8 * (int64_t)bus;
    fd_half_step_to<ANGLE>(wb, br, wb.blk(br), bus, pv, x);
}

// The top of the tree (the LDS tail's levels) of a factored matrix, copied
// into LDS once per launch: (w, u) per local slot, 1/d per local node.
struct FdTail {
    double2* wu;  // TS
    double* d;    // K
};

__device__ __forceinline__ void fd_tail_load(const DevSym& S, const double* m, const FdTail& t)
{
    const double2* sl = reinterpret_cast<const double2*>(m + S.fd_lu);
    for (int i = threadIdx.x; i < S.tail_slots; i += blockDim.x) t.wu[i] = sl[S.t_slot[3 * i].x];
    for (int i = threadIdx.x; i < S.tail_nodes; i += blockDim.x) t.d[i] = m[S.t_node[3 * i].x];
}

// Forward substitution of the tail levels in LDS on component comp: each
// tail node first takes b_j and the terms of its descendants outside the
// tail (global lists, all nodes at once), then the tail levels go upward
// with the local lists.  y of the tail stays in sy for the backward sweep.
template <bool VL>
__device__ __forceinline__ void fd_forward_tail(const DevSym& S, const double* m, const FdTail& t,
                                                double* sy, const View& wb, int64_t rhs,
                                                int comp, double* xv)
{
    const double2* sl = reinterpret_cast<const double2*>(m + S.fd_lu);
    for (int jl = threadIdx.x; jl < S.tail_nodes; jl += blockDim.x) {
        const int4 a = S.t_node[3 * jl], b = S.t_node[3 * jl + 1];
        double z = *wb.at(rhs + 2 * (int64_t)a.x + comp);
        const int r1 = b.z;
        int r = b.y;
        int2 e[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) e[k] = S.t_rl[r + k < r1 ? r + k : 0];
        for (; r < r1; r += 4) {
            double w[4], y[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                w[k] = sl[e[k].y].x;
                y[k] = fd_x<VL>(xv, wb, rhs, comp, e[k].x);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) e[k] = S.t_rl[r + 4 + k < r1 ? r + 4 + k : 0];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (r + k < r1) z = fma(-w[k], y[k], z);
        }
        sy[jl] = z;
    }
    __syncthreads();
    const int nT = S.nlev - S.tail_level, KC = S.tail_clique;
    for_tail_pf(S, 0, nT - KC, true, [&](int jl, const int4&, const int4& b, const int4&,
                                         int lane, int g) {
        double z = 0.0;
        for (int r = b.z + lane; r < b.w; r += g) {
            const int2 e = S.t_rl[r];
            z = fma(t.wu[e.y].x, sy[e.x], z);
        }
        if (g > 1) z = gsum(z, g);
        if (lane == 0) sy[jl] = t.d[jl] * (sy[jl] - z);
    });
    if (KC > 0) {
        // the clique (every node adjacent to all above it): first the terms of
        // the tail nodes below it, all clique nodes at once; then the clique
        // column by column on the first wavefront (no workgroup barriers)
        const int kf = S.tail_nodes - KC;
        for (int c = threadIdx.x; c < KC; c += blockDim.x) {
            const int jl = kf + c;
            const int4 b = S.t_node[3 * jl + 1], cm = S.t_node[3 * jl + 2];
            double z = 0.0;
            for (int r = b.z; r < cm.x; ++r) {
                const int2 e = S.t_rl[r];
                z = fma(t.wu[e.y].x, sy[e.x], z);
            }
            sy[jl] -= z;
        }
        __syncthreads();
        if (threadIdx.x < kWave) {
            const int c0 = S.t_node[3 * kf].w;
            for (int q = 0; q < KC; ++q) {
                const double yq = t.d[kf + q] * sy[kf + q];
                for (int k = q + 1 + threadIdx.x; k < KC; k += kWave)
                    sy[kf + k] = fma(-t.wu[clique_slot(c0, KC, q, k)].x, yq, sy[kf + k]);
                if (threadIdx.x == 0) sy[kf + q] = yq;
                wave_sync();
            }
        }
        __syncthreads();
    }
}

// Backward substitution of the tail levels in LDS, downward; then, in one
// parallel pass (so that no level waits for a bus-record load), each tail x
// is written to the rhs for the levels below and its bus takes the half step.
template <bool ANGLE, bool VL>
__device__ __forceinline__ void fd_backward_tail(const DevSym& S, const FdTail& t, double* sy,
                                                 const View& wb, int64_t rhs, int64_t bus_off,
                                                 const PvMask& pv, double* xv)
{
    const int comp = ANGLE ? 0 : 1;
    const int nT = S.nlev - S.tail_level, KC = S.tail_clique;
    if (KC > 0) {
        // the clique first, column by column on the first wavefront: once x_q
        // is final, y_k -= u_kq x_q for every clique node k below q
        if (threadIdx.x < kWave) {
            const int kf = S.tail_nodes - KC, c0 = S.t_node[3 * kf].w;
            for (int q = KC - 1; q > 0; --q) {
                const double xq = sy[kf + q];
                for (int k = threadIdx.x; k < q; k += kWave)
                    sy[kf + k] = fma(-t.wu[clique_slot(c0, KC, k, q)].y, xq, sy[kf + k]);
                wave_sync();
            }
        }
        __syncthreads();
    }
    for_tail_pf(S, 0, nT - KC, false, [&](int jl, const int4& a, const int4& b, const int4&,
                                          int lane, int g) {
        double s = 0.0;
        for (int q = a.w + lane; q < b.x; q += g) s = fma(t.wu[q].y, sy[S.t_slot[3 * q].y], s);
        if (g > 1) s = gsum(s, g);
        if (lane == 0) sy[jl] -= s;
    });
    __syncthreads();
    for (int jl = threadIdx.x; jl < S.tail_nodes; jl += blockDim.x) {
        const int4 a = S.t_node[3 * jl];
        const double x = sy[jl];
        fd_x<VL>(xv, wb, rhs, comp, a.x) = x;
        fd_half_step<ANGLE>(wb, bus_off, a.y, pv, x);
    }
    __syncthreads();
}

// Backward substitution x_j = y_j - sum_{k in S(j)} u_jk x_k, levels
// downward, and the half step at bus(j); four slots per lane per batch with
// the next batch's indices in flight.
template <bool ANGLE, bool VL>
__device__ __forceinline__ void fd_backward(const DevSym& S, const double* m, const View& wb,
                                            int64_t rhs, int64_t bus_off, const PvMask& pv,
                                            int l1, double* xv)
{
    const double2* sl = reinterpret_cast<const double2*>(m + S.fd_lu);
    const int comp = ANGLE ? 0 : 1;
    for_nodes(S, 0, l1, false, [&](int, const NodeRec& rec, int lane, int g) {
        const int s1 = rec.b.y;
        const double yj = fd_x<VL>(xv, wb, rhs, comp, rec.a.x);
        // absent entries are not loaded (skipped when no lane needs them)
        int s = rec.b.x + lane;
        int kk[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            kk[k] = 0;
            if (s + k * g < s1) kk[k] = S.Li[s + k * g];
        }
        double a = 0.0;
        for (; s < s1; s += 4 * g) {
            double u[4], x[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                u[k] = 0.0;
                x[k] = 0.0;
                if (s + k * g < s1) {
                    u[k] = sl[s + k * g].y;
                    x[k] = fd_x<VL>(xv, wb, rhs, comp, kk[k]);
                }
            }
            const int sn = s + 4 * g;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (sn + k * g < s1) kk[k] = S.Li[sn + k * g];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (s + k * g < s1) a = fma(u[k], x[k], a);
        }
        if (g > 1) a = gsum(a, g);
        if (lane == 0) {
            const double xj = yj - a;
            fd_x<VL>(xv, wb, rhs, comp, rec.a.x) = xj;
            fd_half_step<ANGLE>(wb, bus_off, rec.a.y, pv, xj);
        }
    });
}

// The fast decoupled iteration of one case (one workgroup): mismatch, angle
// half step with B', mismatch, magnitude half step with B'', until max|F| <
// tol; iters counts angle half steps and max_iter bounds them.  VL: the
// half step's work vector in LDS (after the tail of the half step's matrix).
template <bool VL>
__device__ void fdpf_case(const DevSym& S, const double* yv, const int8_t* type,
                          const double* Psp, const double* Qsp, double* Vm, double* Va,
                          const View& wb, const double* m1, const double* m2, double tol,
                          int max_iter, int32_t* o_iters, double* o_norm, int32_t* o_status)
{
    // LDS: PV mask, then either (ef_lds = 0) the (w, u) of the B' and B''
    // tails | 1/d of both | tail y, loaded once; or the (e, f) copy of the
    // mismatch pass, over which the tail of the matrix of the half step
    // (w, u | 1/d | y) is loaded after each mismatch
    uint32_t* fd_pv = reinterpret_cast<uint32_t*>(pf_smem);
    double* lds = pf_smem + ((((S.n + 63) / 64) + 1) & ~1);  // mask: 8 bytes per 64 buses
    const int K = S.tail_nodes, TS = S.tail_slots;
    const bool efl = S.ef_lds != 0;
    const FdTail t1{reinterpret_cast<double2*>(lds), lds + (efl ? 2 : 4) * TS};
    const FdTail t2 = efl ? t1 : FdTail{reinterpret_cast<double2*>(lds + 2 * TS), lds + 4 * TS + K};
    double* sy = efl ? lds + 2 * TS + K : lds + 4 * TS + 2 * K;
    double* xv = lds + 2 * TS + 2 * K;  // VL only
    const bool tail = K > 0;
    const int lg = tail ? S.tail_level : S.nlev;  // levels swept in global memory
    if (tail && !efl) {
        fd_tail_load(S, m1, t1);
        fd_tail_load(S, m2, t2);
    }
    const Off o = ws_off(S);
    for (int i = threadIdx.x; i < S.n; i += blockDim.x) {
        double sn, cs;
        const double vm = Vm[i], va = Va[i];
        sincos(va, &sn, &cs);
        wb.put(o.BUS + 8 * (int64_t)i, {vm * cs, vm * sn, vm, va});
    }
    pv_fill_at(fd_pv, S, type);
    __syncthreads();
    const PvMask pvm{fd_pv};
    const EFView ef{wb, o.BUS};
    int it = 0, half = 0, st = ST_NOT_CONVERGED;
    double nrm = 0.0;
    for (;;) {
        double mx = 0.0;
        int nan = 0;
        if (efl) {
            const EFLds efs{reinterpret_cast<double2*>(lds)};
            for (int i = threadIdx.x; i < S.n; i += blockDim.x)
                efs.s[i] = wb.v2(o.BUS + 8 * (int64_t)i);
            __syncthreads();
            mismatch_pass<true>(S, yv, efs, wb, o, pvm, Psp, Qsp, mx, nan);
        } else {
            mismatch_pass<true>(S, yv, ef, wb, o, pvm, Psp, Qsp, mx, nan);
        }
        int any_nan = 0;
        nrm = block_max(mx, nan, any_nan);
        if (any_nan || !isfinite(nrm)) {
            st = ST_NONFINITE;
            break;
        }
        if (nrm < tol) {
            st = ST_OK;
            break;
        }
        if (efl && tail && (half != 0 || it < max_iter)) {
            fd_tail_load(S, half == 0 ? m1 : m2, t1);
            __syncthreads();
        }
        if (half == 0) {
            if (it >= max_iter) {
                st = ST_NOT_CONVERGED;
                break;
            }
            fd_forward<VL>(S, m1, wb, o.RHS, 0, lg, xv);
            if (tail) {
                fd_forward_tail<VL>(S, m1, t1, sy, wb, o.RHS, 0, xv);
                fd_backward_tail<true, VL>(S, t1, sy, wb, o.RHS, o.BUS, pvm, xv);
            }
            fd_backward<true, VL>(S, m1, wb, o.RHS, o.BUS, pvm, lg, xv);
            ++it;
        } else {
            fd_forward<VL>(S, m2, wb, o.RHS, 1, lg, xv);
            if (tail) {
                fd_forward_tail<VL>(S, m2, t2, sy, wb, o.RHS, 1, xv);
                fd_backward_tail<false, VL>(S, t2, sy, wb, o.RHS, o.BUS, pvm, xv);
            }
            fd_backward<false, VL>(S, m2, wb, o.RHS, o.BUS, pvm, lg, xv);
        }
        half ^= 1;
    }
    for (int i = threadIdx.x; i < S.n; i += blockDim.x) {
        const Blk r = wb.blk(o.BUS + 8 * (int64_t)i);
        Vm[i] = r.c;
        Va[i] = r.d;
    }
    if (threadIdx.x == 0) {
        if (o_iters) *o_iters = it;
        if (o_norm) *o_norm = nrm;
        if (o_status) *o_status = st;
    }
}


}  // namespace


// Fast decoupled matrices of B cases: B' then B'' (fd_mat doubles each) in
// the scalar filled layout, lower and upper values equal.
__global__ void k_fd_matrices(DevSym S, const double* __restrict__ r,
                              const double* __restrict__ x, const double* __restrict__ b,
                              int64_t bstride, const double* __restrict__ ysh,
                              int64_t sh_stride, const int8_t* __restrict__ type,
                              int64_t type_stride, double* __restrict__ mat, int64_t mstride)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (p >= S.fd_lu) return;
    const double* rc = r + c * bstride;
    const double* xc = x + c * bstride;
    const double* bc = b + c * bstride;
    const int8_t* tc = type + c * type_stride;
    double* m1 = mat + c * mstride;
    double* m2 = m1 + S.fd_mat;
    if (p >= S.nn) {  // padding of the d sections
        m1[p] = 0.0;
        m2[p] = 0.0;
        return;
    }
    const bool pvj = tc[S.perm[p]] == T_PV;
    // B'' = -Im(Y): the bus shunt's susceptance comes off the diagonal
    const double bsh = ysh ? ysh[c * sh_stride + 2 * (int64_t)S.perm[p] + 1] : 0.0;
    m1[p] = fd_entry<false>(S, S.ydiag[p], true, rc, xc, bc);
    m2[p] = pvj ? 1.0 : fd_entry<true>(S, S.ydiag[p], true, rc, xc, bc) - bsh;
    double2* s1 = reinterpret_cast<double2*>(m1 + S.fd_lu);
    double2* s2 = reinterpret_cast<double2*>(m2 + S.fd_lu);
    for (int s = S.Lp[p]; s < S.Lp[p + 1]; ++s) {
        const int q = S.ylo[s];
        const bool pvk = tc[S.perm[S.Li[s]]] == T_PV;
        const double v1 = q < 0 ? 0.0 : fd_entry<false>(S, q, false, rc, xc, bc);
        const double v2 = (q < 0 || pvj || pvk) ? 0.0 : fd_entry<true>(S, q, false, rc, xc, bc);
        s1[s] = make_double2(v1, v1);
        s2[s] = make_double2(v2, v2);
    }
}

// In-place LDL^T of B' and B'' of case blockIdx.x, level by level.
// Two workgroups per case, one per matrix (B' and B'' are independent).  The
// status is set to OK by k_fill_status beforehand; a workgroup that meets a
// zero pivot stores ST_ZERO_PIVOT (both may, with the same value).
__global__ __launch_bounds__(kLevelThreads) void k_fd_factor(DevSym S, double* mat,
                                                             int64_t mstride, int32_t* status)
{
    __shared__ int s_bad;
    const int c = blockIdx.x >> 1, which = blockIdx.x & 1;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    double* m = mat + c * mstride + which * S.fd_mat;
    for_nodes(S, 0, S.nlev, true, [&](int, const NodeRec& rec, int lane, int g) {
        fd_factor_node(S, rec, lane, g, m, &s_bad);
    });
    __syncthreads();
    if (threadIdx.x == 0 && status && s_bad) status[c] = ST_ZERO_PIVOT;
}

__global__ void k_fill_status(int B, int32_t* status, int32_t v)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < B) status[c] = v;
}

__global__ __launch_bounds__(kLevelThreads) void k_fdpf(DevSym S, NewtonArgs a,
                                                        const double* mat, int64_t mstride)
{
    const int c = blockIdx.x;
    View wb;
    wb.base = a.ws + c * a.ws_stride;
    wb.lane = 0;
    wb.sh = 2;
    wb.cs = 2;
    const double* m1 = mat + c * mstride;
    // the work vector fits in LDS after one matrix's tail, within the (e, f) copy
    const bool vl = S.ef_lds != 0 &&
                    16 * ((int64_t)S.tail_slots + S.tail_nodes) + 8 * (int64_t)S.nn <= S.ef_lds;
    auto run = [&](auto tag) {
        fdpf_case<decltype(tag)::value>(
            S, a.yval + c * a.y_stride, a.type + c * a.type_stride, a.Psp + c * a.inj_stride,
            a.Qsp + c * a.inj_stride, a.Vm + c * a.v_stride, a.Va + c * a.v_stride, wb, m1,
            m1 + S.fd_mat, a.tol, a.max_iter, a.iters ? a.iters + c : nullptr,
            a.norm ? a.norm + c : nullptr, a.status ? a.status + c : nullptr);
    };
    if (vl) run(std::true_type{});
    else run(std::false_type{});
}

// Branch flows (Sec. II-A: post-convergence, edge by edge): pi-model with
// series y = 1/(r + jx) and charging b, I_ft = (y + jb/2) V_f - y V_t,
// S_ft = V_f conj(I_ft), and the same from the other end.
__global__ void k_branch_flows(int m, const int32_t* __restrict__ from,
                               const int32_t* __restrict__ to, const double* __restrict__ r,
                               const double* __restrict__ x, const double* __restrict__ b,
                               int64_t bstride, const double* __restrict__ Vm,
                               const double* __restrict__ Va, int64_t vstride, double* Pft,
                               double* Qft, double* Ptf, double* Qtf, int64_t ostride)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (e >= m) return;
    const int fb = from[e], tb = to[e];
    const double rr = r[c * bstride + e], xx = x[c * bstride + e], hb = b[c * bstride + e] / 2.0;
    const double den = rr * rr + xx * xx;
    const double yg = rr / den, yb = -xx / den;
    const double* vm = Vm + c * vstride;
    const double* va = Va + c * vstride;
    double sf, cf, st, ct;
    sincos(va[fb], &sf, &cf);
    sincos(va[tb], &st, &ct);
    const double ef = vm[fb] * cf, ff = vm[fb] * sf, et = vm[tb] * ct, ft = vm[tb] * st;
    // I_ft = (yg + j(yb + hb)) V_f - (yg + j yb) V_t, and symmetrically
    const double ifr = yg * ef - (yb + hb) * ff - (yg * et - yb * ft);
    const double ifi = yg * ff + (yb + hb) * ef - (yg * ft + yb * et);
    const double itr = yg * et - (yb + hb) * ft - (yg * ef - yb * ff);
    const double iti = yg * ft + (yb + hb) * et - (yg * ff + yb * ef);
    const int64_t o = c * ostride + e;
    Pft[o] = ef * ifr + ff * ifi;  // V conj(I)
    Qft[o] = ff * ifr - ef * ifi;
    Ptf[o] = et * itr + ft * iti;
    Qtf[o] = ft * itr - et * iti;
}


namespace {

// Dynamic LDS of the fast decoupled kernel: PV mask (rounded to 16 bytes),
// then (w, u) of both matrices' tails, 1/d of both, and the tail's y.
size_t fd_lds_bytes(const HostSym& h)
{
    const size_t mask = ((pv_mask_bytes(h.n) + 15) / 16) * 16;
    if (h.ef_lds)  // (e, f) copy, and one matrix's tail at a time over it
        return mask + std::max((size_t)h.ef_lds,
                               8 * (2 * (size_t)h.tail_slots + 2 * (size_t)h.tail_nodes));
    return mask + 8 * (4 * (size_t)h.tail_slots + 3 * (size_t)h.tail_nodes);
}

// Raises the dynamic-LDS limit of the fast decoupled kernel to what the device
// allows minus its static LDS (failures keep the default limit).
void allow_big_lds_fdpf()
{
    static bool done = false;
    if (done) return;
    done = true;
    int dev = 0, lds_max = 0;
    hipFuncAttributes fa{};
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) ==
            hipSuccess &&
        hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(&k_fdpf)) == hipSuccess) {
        const int dyn = lds_max - (int)fa.sharedSizeBytes;
        if (dyn > 0)
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fdpf),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    }
    (void)hipGetLastError();
}

}  // namespace

extern "C" {
int pf_fdpf_matrices(const pf_symbolic s, int B, const double* d_r, const double* d_x,
                     const double* d_b, int64_t branch_stride, const double* d_ysh,
                     int64_t ysh_stride, const int8_t* d_type, int64_t type_stride,
                     double* d_mat, int64_t mat_stride, void* stream)
{
    if (!ready(s, "pf_fdpf_matrices")) return PF_E_INVALID;
    if (B < 0 || B > 65535 || !d_r || !d_x || !d_b || !d_type || !d_mat || (mat_stride & 7) ||
        branch_stride < 0 || ysh_stride < 0)
        return fail(PF_E_INVALID, "pf_fdpf_matrices: bad arguments");
    if (d_ysh && (ysh_stride & 1 || (B > 1 && ysh_stride != 0 && ysh_stride < 2 * s->h.n)))
        return fail(PF_E_INVALID, "pf_fdpf_matrices: ysh_stride must be 0 or even and >= 2*n");
    if (reinterpret_cast<uintptr_t>(d_mat) & 15)
        return fail(PF_E_WORKSPACE, "pf_fdpf_matrices: d_mat must be 16-byte aligned");
    if (B > 1 && mat_stride < 2 * s->h.fd_mat())
        return fail(PF_E_WORKSPACE, "pf_fdpf_matrices: mat_stride < fd_mat_doubles");
    if (!shared_stride_ok(B, branch_stride, s->h.m) || !shared_stride_ok(B, type_stride, s->h.n))
        return fail(PF_E_WORKSPACE, "pf_fdpf_matrices: a stride is too small or negative");
    if (B == 0) return PF_OK;
    dim3 grid((unsigned)((s->h.fd_lu() + 255) / 256), B);
    hipLaunchKernelGGL(k_fd_matrices, grid, dim3(256), 0, as_stream(stream), s->h.dev, d_r, d_x,
                       d_b, branch_stride, d_ysh, ysh_stride, d_type, type_stride, d_mat,
                       mat_stride);
    return launch_check("pf_fdpf_matrices");
}

int pf_fdpf_factor(const pf_symbolic s, int B, double* d_mat, int64_t mat_stride,
                   int32_t* d_status, void* stream)
{
    if (!ready(s, "pf_fdpf_factor")) return PF_E_INVALID;
    if (B < 0 || !d_mat || (mat_stride & 7))
        return fail(PF_E_INVALID, "pf_fdpf_factor: bad arguments");
    if (reinterpret_cast<uintptr_t>(d_mat) & 15)
        return fail(PF_E_WORKSPACE, "pf_fdpf_factor: d_mat must be 16-byte aligned");
    if (B > 1 && mat_stride < 2 * s->h.fd_mat())
        return fail(PF_E_WORKSPACE, "pf_fdpf_factor: mat_stride < fd_mat_doubles");
    if (B == 0) return PF_OK;
    if (d_status)
        hipLaunchKernelGGL(k_fill_status, dim3((B + 255) / 256), dim3(256), 0, as_stream(stream),
                           B, d_status, (int32_t)ST_OK);
    hipLaunchKernelGGL(k_fd_factor, dim3(2 * B), dim3(launch_threads(s->h, B)), 0,
                       as_stream(stream), s->h.dev, d_mat, mat_stride, d_status);
    return launch_check("pf_fdpf_factor");
}

int pf_fdpf(const pf_symbolic s, int B, const double* d_yval, int64_t y_stride,
            const int8_t* d_type, int64_t type_stride, const double* d_Psp, const double* d_Qsp,
            int64_t inj_stride, double* d_Vm, double* d_Va, int64_t v_stride,
            const double* d_mat, int64_t mat_stride, double tol, int max_iter, double* d_ws,
            int64_t ws_stride, int32_t* d_iters, double* d_norm, int32_t* d_status,
            void* stream)
{
    if (!ready(s, "pf_fdpf")) return PF_E_INVALID;
    if (B < 0 || max_iter < 0 || !(tol >= 0.0) || !d_yval || !d_type || !d_Psp || !d_Qsp ||
        !d_Vm || !d_Va || !d_mat || !d_ws || (mat_stride & 7))
        return fail(PF_E_INVALID, "pf_fdpf: bad arguments");
    if (B > 1 && v_stride < s->h.n) return fail(PF_E_WORKSPACE, "pf_fdpf: v_stride too small");
    if (!shared_stride_ok(B, y_stride, 2 * (int64_t)s->h.ycol.size()) ||
        !shared_stride_ok(B, type_stride, s->h.n) || !shared_stride_ok(B, inj_stride, s->h.n) ||
        !shared_stride_ok(B, mat_stride, 2 * s->h.fd_mat()))
        return fail(PF_E_WORKSPACE, "pf_fdpf: a stride is too small or negative");
    if (ws_stride < s->h.fd_ws_doubles() || (ws_stride & 7))
        return fail(PF_E_WORKSPACE,
                    "pf_fdpf: ws_stride must be >= fd_ws_doubles, a multiple of 8");
    if ((reinterpret_cast<uintptr_t>(d_ws) & 15) || (reinterpret_cast<uintptr_t>(d_mat) & 15))
        return fail(PF_E_WORKSPACE, "pf_fdpf: d_ws and d_mat must be 16-byte aligned");
    if (B == 0) return PF_OK;
    NewtonArgs a{d_yval, y_stride, d_type, type_stride, d_Psp, d_Qsp, inj_stride, d_Vm, d_Va,
                 v_stride, d_ws, ws_stride, tol, max_iter, 0, 1, B, d_iters, d_norm, d_status};
    allow_big_lds_fdpf();
    hipLaunchKernelGGL(k_fdpf, dim3(B), dim3(launch_threads(s->h, B)),
                       fd_lds_bytes(s->h), as_stream(stream), s->h.dev, a, d_mat, mat_stride);
    return launch_check("pf_fdpf");
}

int pf_branch_flows(const pf_symbolic s, int B, const double* d_r, const double* d_x,
                    const double* d_b, int64_t branch_stride, const double* d_Vm,
                    const double* d_Va, int64_t v_stride, double* d_Pft, double* d_Qft,
                    double* d_Ptf, double* d_Qtf, int64_t out_stride, void* stream)
{
    if (!ready(s, "pf_branch_flows")) return PF_E_INVALID;
    if (B < 0 || B > 65535 || !d_r || !d_x || !d_b || !d_Vm || !d_Va || !d_Pft || !d_Qft ||
        !d_Ptf || !d_Qtf)
        return fail(PF_E_INVALID, "pf_branch_flows: bad arguments");
    if (B > 1 && (v_stride < s->h.n || out_stride < s->h.m))
        return fail(PF_E_WORKSPACE, "pf_branch_flows: stride too small");
    if (!shared_stride_ok(B, branch_stride, s->h.m))
        return fail(PF_E_WORKSPACE, "pf_branch_flows: branch_stride too small or negative");
    if (B == 0 || s->h.m == 0) return PF_OK;
    dim3 grid((s->h.m + 255) / 256, B);
    hipLaunchKernelGGL(k_branch_flows, grid, dim3(256), 0, as_stream(stream), s->h.m, s->d_from,
                       s->d_to, d_r, d_x, d_b, branch_stride, d_Vm, d_Va, v_stride, d_Pft, d_Qft,
                       d_Ptf, d_Qtf, out_stride);
    return launch_check("pf_branch_flows");
}

}  // extern "C"
