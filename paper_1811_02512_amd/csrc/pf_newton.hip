// libpf Newton-Raphson path: admittance matrix, mismatch, Jacobian, block
// LDU, solves, the fused Newton kernel, the adjoint and multi-pattern
// batches (kernels and their C ABI entry points).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <type_traits>
#include <vector>

#include "pf.h"
#include "pf_device.h"
#include "pf_host.h"

using namespace pf::abi;

namespace {

// The whole Newton-Raphson loop of one case, run by one workgroup (OneGroup)
// or by every workgroup of a cooperative launch (Spread: the loops over
// buses and the levels below the LDS tail are shared out, the tail runs on
// workgroup 0).  The case's voltages and injections are copied into its bus
// records first and the solution copied back at the end.
template <class P>
__device__ __forceinline__ void newton_case(const P& par, const DevSym& S, const double* yv,
                                            const int8_t* type, const double* Psp,
                                            const double* Qsp, double* Vm, double* Va,
                                            const View& w, const View& wb, double tol,
                                            int max_iter, int flags, int32_t* o_iters,
                                            double* o_norm, int32_t* o_status, int32_t* o_pivot)
{
    __shared__ int s_bad;
    constexpr bool kOne = !P::kSpread;
    int* bad = &s_bad;
    if constexpr (P::kSpread) bad = par.marker();
    const bool lead = par.rank() == 0;
    // this thread's first bus and the stride of the loops over buses
    auto t0 = [&]() { return par.rank() * (int)blockDim.x + (int)threadIdx.x; };
    auto ts = [&]() { return par.size() * (int)blockDim.x; };
    const Off o = ws_off(S);
    // the groups of a spread batch of grids: this workgroup's subtrees
    // below the cut
    int k0 = 0, k1 = 0;
    if constexpr (P::kSub) sub_share(S, par, k0, k1);
    for (int i = t0(); i < S.n; i += ts()) {
        double sn, cs;
        const double vm = Vm[i], va = Va[i];
        sincos(va, &sn, &cs);
        wb.put(o.BUS + 8 * (int64_t)i, {vm * cs, vm * sn, vm, va});
    }
    pv_fill(S, type);
    if (kOne && threadIdx.x == 0) s_bad = kNoPivot;
    par.sync();
    // the zero-pivot marker; in a spread launch thread 0 reads it and hands
    // it to its workgroup, so that every thread of a workgroup takes the
    // same branch even if other workgroups have lost step (called by every
    // thread of the workgroup)
    __shared__ int s_mark;
    auto marker = [&]() {
        if constexpr (P::kSpread) {
            if (threadIdx.x == 0)
                s_mark = __hip_atomic_load(bad, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
            const int v = s_mark;
            __syncthreads();
            return v;
        } else {
            return s_bad;
        }
    };
    // the tail's results are read by the other workgroups of a spread launch
    // only after a grid barrier (one workgroup's own barriers order them);
    // the tail's factorisation is entered by every workgroup (they share its
    // first pass), its backward substitution by workgroup 0 alone
    auto tail_done = [&]() {
        if constexpr (P::kSpread) par.sync();
    };
    const PvMask pvm{pv_words(S)};
    // one workgroup: the global levels of the factorisation sweep read
    // neighbours' (e, f) from the LDS copy the mismatch pass just made (the
    // tail reuses that LDS afterwards and reads them from the bus records),
    // and the backward sweep keeps x in that LDS too (free again once the
    // tail's backward substitution has read its values)
    const bool efl = kOne && S.ef_lds;
    const SrcState src{yv, pvm, wb, o.BUS,
                       efl ? reinterpret_cast<const double2*>(pf_smem) : nullptr};
    double2* const xs = (efl && S.tail_nodes <= 4 * (int)blockDim.x)
                            ? reinterpret_cast<double2*>(pf_smem)
                            : nullptr;
    const EFView ef{wb, o.BUS};
    const bool tail = S.tail_nodes > 0;
    int it = 0, st = ST_NOT_CONVERGED;
    double nrm = 0.0;
    for (;;) {
        double mx = 0.0;
        int nan = 0;
        if (efl) {
            // every bus's (e, f) into LDS (free until the tail), so that the
            // admittance rows' voltages are LDS reads
            const EFLds el{reinterpret_cast<double2*>(pf_smem)};
            for (int i = threadIdx.x; i < S.n; i += blockDim.x)
                el.s[i] = wb.v2(o.BUS + 8 * (int64_t)i);
            __syncthreads();
            mismatch_pass<false, EFLds, 4>(S, yv, el, wb, o, pvm, Psp, Qsp, mx, nan);
        } else {
            mismatch_pass<false>(S, yv, ef, wb, o, pvm, Psp, Qsp, mx, nan, t0(), ts());
        }
        int any_nan = 0;
        nrm = block_max(mx, nan, any_nan);
        if constexpr (P::kSpread) {
            // every workgroup's maximum and NaN flag into this iteration's
            // slots; after the barrier all read the same norm
            const int sl = it & 1;
            if (threadIdx.x == 0) {
                if (any_nan)
                    __hip_atomic_fetch_or(par.flags + 2 + sl, 1, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_max(par.maxbits + sl, (uint64_t)__double_as_longlong(nrm),
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            par.sync();
            // thread 0 reads the norm for its workgroup (as the marker)
            __shared__ double s_nrm;
            __shared__ int s_nan;
            if (threadIdx.x == 0) {
                s_nan = __hip_atomic_load(par.flags + 2 + sl, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
                s_nrm = __longlong_as_double((long long)__hip_atomic_load(
                    par.maxbits + sl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                // the other slots were last read before the previous
                // iteration's later barriers: clear them for the next one
                if (lead) {
                    __hip_atomic_store(par.flags + 3 - sl, 0, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(par.maxbits + 1 - sl, (uint64_t)0, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            __syncthreads();
            any_nan = s_nan;
            nrm = s_nrm;
            __syncthreads();
        }
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
        auto fwd = [&](int x, const NodeRec& r, int lane, int g) {
            factor_node<SrcState, true, false>(S, src, x, r, lane, g, w, o.LU, wb, o.RHS, bad);
        };
        int lc = 0;  // first level shared among the workgroups
        if constexpr (P::kSub) {
            if (S.sub_cut > 0) {
                for_sub_levels(S, k0, k1, 0, S.sub_cut, true, fwd);
                par.sync();
                lc = S.sub_cut;
            }
        }
        for_nodes(par, S, lc, S.tail_level, true, fwd);
        if (tail) {
            tail_factor<SrcState, true, false>(S, src, w, o.LU, wb, o.RHS, bad, par);
            tail_done();
        }
        if (marker() != kNoPivot) {
            st = ST_ZERO_PIVOT;
            break;
        }
        auto back = [&](int, const NodeRec& r, int lane, int g) {
            back_node<true>(S, r, lane, g, w, o.LU, wb, o.RHS, o.BUS, pvm, xs);
        };
        int lw = S.tail_level;
        if constexpr (P::kSpread) lw = par.back_lo;
        if (tail || lw < S.tail_level) {
            if (lead) {
                if (tail) tail_backward<true>(S, wb, o.RHS, o.BUS, pvm, xs);
                if constexpr (P::kSpread) for_nodes(OneGroup{}, S, lw, S.tail_level, false, back);
            }
            tail_done();
        }
        // below min(cut, lw): each workgroup its own subtrees, top-down
        int lb = 0;
        if constexpr (P::kSub) lb = S.sub_cut < lw ? S.sub_cut : lw;
        for_nodes(par, S, lb, lw, false, back);
        if constexpr (P::kSub) {
            if (lb > 0) {
                for_sub_levels(S, k0, k1, 0, lb, false, back);
                par.sync();
            }
        }
        ++it;
    }
    if ((flags & PF_NEWTON_KEEP_FACTORS) && st == ST_OK) {
        auto keep = [&](int x, const NodeRec& r, int lane, int g) {
            factor_node<SrcState, false, true>(S, src, x, r, lane, g, w, o.LU, wb, o.RHS, bad);
        };
        int lc = 0;
        if constexpr (P::kSub) {
            if (S.sub_cut > 0) {
                for_sub_levels(S, k0, k1, 0, S.sub_cut, true, keep);
                par.sync();
                lc = S.sub_cut;
            }
        }
        for_nodes(par, S, lc, S.tail_level, true, keep);
        if (tail) {
            tail_factor<SrcState, false, true>(S, src, w, o.LU, wb, o.RHS, bad, par);
            tail_done();
        }
        if (marker() != kNoPivot) st = ST_ZERO_PIVOT;
    }
    for (int i = t0(); i < S.n; i += ts()) {
        const Blk r = wb.blk(o.BUS + 8 * (int64_t)i);
        Vm[i] = r.c;
        Va[i] = r.d;
    }
    const int bad_at = marker();
    if (lead && threadIdx.x == 0) {
        if constexpr (P::kSpread) {
            if (par.aborted()) st = PF_E_HIP;
        }
        if (o_iters) *o_iters = it;
        if (o_norm) *o_norm = nrm;
        if (o_status) *o_status = st;
        if (o_pivot) *o_pivot = bad_at == kNoPivot ? -1 : S.level_nodes[bad_at];
    }
}

// Jacobian assembly straight from polar voltages (standalone kernel).
struct AsmPolar {
    const DevSym* S;
    const double* yv;
    const int8_t* type;
    const double* Vm;
    EFPolar ef;
    __device__ __forceinline__ Blk diag(int j) const
    {
        const int bus = S->perm[j];
        const double2 y = reinterpret_cast<const double2*>(yv)[S->ydiag[j]];
        double p, q;
        injection(*S, yv, ef, bus, p, q);
        return jac_diag(y.x, y.y, p, q, Vm[bus], type[bus] == T_PV);
    }
    __device__ __forceinline__ void off(int j, int s, Blk& lo, Blk& up) const
    {
        const int ylo = S->ylo[s];
        if (ylo < 0) {
            lo = bzero();
            up = bzero();
            return;
        }
        const int bj = S->perm[j], bk = S->perm[S->Li[s]];
        double ej, fj, ek, fk;
        ef.get(bj, ej, fj);
        ef.get(bk, ek, fk);
        const bool pj = type[bj] == T_PV, pk = type[bk] == T_PV;
        const double2 yl = reinterpret_cast<const double2*>(yv)[ylo];
        const double2 yu = reinterpret_cast<const double2*>(yv)[S->yup[s]];
        lo = jac_off(yl.x, yl.y, ek, fk, ej, fj, Vm[bj], pk, pj);
        up = jac_off(yu.x, yu.y, ej, fj, ek, fk, Vm[bk], pj, pk);
    }
};

}  // namespace

// ===========================================================================
// kernels
// ===========================================================================
// Threads per admittance row in the assembly kernels.
constexpr int kYbusLanes = 4;

// Row i of the admittance matrix (FormMatrixA): the diagonal starts from the
// bus's shunt (ysh: (g, b) of bus i, or null), then every branch in the
// entry's list adds y + jb/2 (diagonal) or -y (off-diagonal), in list order.
// Entries q0 + sub, q0 + sub + nsub, ... of the row are this thread's
// (several threads per row, so that the rows' short chains of dependent
// loads overlap).
__device__ __forceinline__ void ybus_row(const DevSym& S, int i, int sub, int nsub,
                                         const double* __restrict__ rc,
                                         const double* __restrict__ xc,
                                         const double* __restrict__ bcc,
                                         const double2* __restrict__ ysh, double* __restrict__ yc)
{
    for (int q = S.yptr[i] + sub; q < S.yptr[i + 1]; q += nsub) {
        const bool diag = S.ycol[q] == i;
        double G = 0.0, Bv = 0.0;
        if (diag && ysh) {
            const double2 sh = ysh[i];
            G = sh.x;
            Bv = sh.y;
        }
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

__global__ void k_ybus(DevSym S, const double* __restrict__ r, const double* __restrict__ x,
                       const double* __restrict__ bc, int64_t bstride,
                       const double* __restrict__ ysh, int64_t sh_stride,
                       double* __restrict__ yval, int64_t ystride)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = t / kYbusLanes;
    const int c = blockIdx.y;
    if (i >= S.n) return;
    const double2* sh = ysh ? reinterpret_cast<const double2*>(ysh + c * sh_stride) : nullptr;
    ybus_row(S, i, t % kYbusLanes, kYbusLanes, r + c * bstride, x + c * bstride,
             bc + c * bstride, sh, yval + c * ystride);
}

// Case blockIdx.x of a batch of grids; its rows are shared by the gridDim.y
// workgroups of that case (a large grid's rows spread over many CUs).
__global__ void k_ybus_multi(const CaseDesc* __restrict__ descs, const double* __restrict__ r,
                             const double* __restrict__ x, const double* __restrict__ bc,
                             const double* __restrict__ ysh, double* __restrict__ yval)
{
    const CaseDesc& cd = descs[blockIdx.x];
    const DevSym& S = cd.sym;
    const double2* sh = ysh ? reinterpret_cast<const double2*>(ysh) + cd.bus_off : nullptr;
    const int64_t n = (int64_t)S.n * kYbusLanes;
    for (int64_t t = blockIdx.y * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.y * blockDim.x)
        ybus_row(S, (int)(t / kYbusLanes), (int)(t % kYbusLanes), kYbusLanes, r + cd.br_off,
                 x + cd.br_off, bc + cd.br_off, sh, yval + cd.y_off);
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
                           int64_t v_stride, double* vals, int64_t vals_stride, int C)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (j >= S.nn) return;
    const EFPolar ef{Vm + c * v_stride, Va + c * v_stride};
    const AsmPolar A{&S, yval + c * y_stride, type + c * type_stride, Vm + c * v_stride, ef};
    const View w = case_view(vals, vals_stride, C, c);
    const int64_t lu = S.lu_off;
    w.put(4 * (int64_t)j, A.diag(j));
    for (int s = S.Lp[j]; s < S.Lp[j + 1]; ++s) {
        Blk lo, up;
        A.off(j, s, lo, up);
        w.put(lu + 8 * (int64_t)s, lo);
        w.put(lu + 8 * (int64_t)s + 4, up);
    }
}

// SYM: a symmetric matrix; the levels below the LDS tail update the lower
// blocks only (the tail runs the general LDU, exact for it too).
template <bool SYM>
__global__ __launch_bounds__(kLevelThreads) void k_factor(DevSym S, double* vals,
                                                        int64_t vals_stride, int C, int B,
                                                        int32_t* status, int32_t* pivot)
{
    __shared__ int s_bad;
    const int c = case_of_block(blockIdx.x, C, B);
    if (c < 0) return;
    const View w = case_view(vals, vals_stride, C, c);
    const int64_t lu = S.lu_off;
    if (threadIdx.x == 0) s_bad = kNoPivot;
    __syncthreads();
    const SrcLoadT<SYM> src{w, lu};
    for_nodes(S, 0, S.tail_level, true, [&](int x, const NodeRec& r, int lane, int g) {
        factor_node<SrcLoadT<SYM>, false, true, SYM>(S, src, x, r, lane, g, w, lu, w, 0, &s_bad);
    });
    if (S.tail_nodes > 0) tail_factor<SrcLoadT<SYM>, false, true>(S, src, w, lu, w, 0, &s_bad);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (status) status[c] = s_bad != kNoPivot ? ST_ZERO_PIVOT : ST_OK;
        if (pivot) pivot[c] = s_bad == kNoPivot ? -1 : S.level_nodes[s_bad];
    }
}

// transpose = 0: y_j = D_j^-1 (b_j - sum_{i in R(j)} W_ji y_i)  (levels up),
//                x_j = y_j - sum_{k in S(j)} U_jk x_k            (levels down).
// transpose = 1: p_j = g_j - sum_{i in R(j)} U_ij^T p_i           (levels up),
//                l_j = D_j^-T (p_j - sum_{k in S(j)} W_kj^T l_k)  (levels down).
// A node's g lanes take its list entries in strides of g, four per lane per
// step with the step's blocks and x values requested together; absent
// entries of a step are not loaded and add nothing.  LDSX keeps the case's
// whole vector in LDS (nn x 16 bytes) for the two sweeps.
// The up sweep over levels [0, L) of one case on the vector x2 (position
// order, in LDS or global memory), with the factors in view w.
template <bool TRANS>
__device__ __forceinline__ void solve_up(const DevSym& S, const View& w, double2* x2, int L)
{
    const int64_t lu = S.lu_off;
    for_nodes(S, 0, L, true, [&](int, const NodeRec& rec, int lane, int g) {
        const int j = rec.a.x, r0 = rec.a.z, r1 = rec.a.w;
        double z0 = 0.0, z1 = 0.0;
        for (int base = r0 + lane; base < r1; base += 4 * g) {
            int2 e[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                e[k] = make_int2(0, 0);
                if (base + k * g < r1) e[k] = S.rl[base + k * g];
            }
            Blk M[4];
            double2 xv[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                M[k] = bzero();
                xv[k] = make_double2(0.0, 0.0);
                if (base + k * g < r1) {
                    M[k] = w.blk(lu + 8 * (int64_t)e[k].y + (TRANS ? 4 : 0));
                    xv[k] = x2[e[k].x];
                }
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (base + k * g < r1) {
                    if (TRANS) mtvadd(z0, z1, M[k], xv[k].x, xv[k].y);
                    else mvadd(z0, z1, M[k], xv[k].x, xv[k].y);
                }
            }
        }
        if (g > 1) {
            gsum2(z0, z1, g);
        }
        if (lane == 0) {
            const double2 b = x2[j];
            double u0 = b.x - z0, u1 = b.y - z1;
            if (!TRANS) {
                const Blk Di = w.blk(4 * (int64_t)j);
                double y0 = 0.0, y1 = 0.0;
                mvadd(y0, y1, Di, u0, u1);
                u0 = y0;
                u1 = y1;
            }
            x2[j] = make_double2(u0, u1);
        }
    });
}

// The down sweep over levels [0, L), top-down.
template <bool TRANS>
__device__ __forceinline__ void solve_down(const DevSym& S, const View& w, double2* x2, int L)
{
    const int64_t lu = S.lu_off;
    for_nodes(S, 0, L, false, [&](int, const NodeRec& rec, int lane, int g) {
        const int j = rec.a.x, s0 = rec.b.x, s1 = rec.b.y;
        double a0 = 0.0, a1 = 0.0;
        for (int base = s0 + lane; base < s1; base += 4 * g) {
            int kk[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                kk[k] = 0;
                if (base + k * g < s1) kk[k] = S.Li[base + k * g];
            }
            Blk M[4];
            double2 xv[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                M[k] = bzero();
                xv[k] = make_double2(0.0, 0.0);
                if (base + k * g < s1) {
                    M[k] = w.blk(lu + 8 * (int64_t)(base + k * g) + (TRANS ? 0 : 4));
                    xv[k] = x2[kk[k]];
                }
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (base + k * g < s1) {
                    if (TRANS) mtvadd(a0, a1, M[k], xv[k].x, xv[k].y);
                    else mvadd(a0, a1, M[k], xv[k].x, xv[k].y);
                }
            }
        }
        if (g > 1) {
            gsum2(a0, a1, g);
        }
        if (lane == 0) {
            const double2 y = x2[j];
            double u0 = y.x - a0, u1 = y.y - a1;
            if (TRANS) {
                const Blk Di = w.blk(4 * (int64_t)j);
                double l0 = 0.0, l1 = 0.0;
                mtvadd(l0, l1, Di, u0, u1);
                u0 = l0;
                u1 = l1;
            }
            x2[j] = make_double2(u0, u1);
        }
    });
}

// Orders one wavefront's accesses to the vector (LDS, or global memory with
// workgroup-scope fences).
template <bool LDSX>
__device__ __forceinline__ void sync_x()
{
    if (LDSX) {
        wave_sync();
    } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
}

// The clique chain at the top of the tree (KC single-node levels, each node
// adjacent to every node above it; clique node b's higher neighbours are the
// clique nodes above it in order, so the slot of (b; a), a > b, is entry
// a - b - 1 of S(b)) in the two sweeps:
//   transpose = 0: y_a = D_a^-1 (b_a - sum_{i in R(a)} W_ai y_i),
//                  x_a = y_a - sum_{c > a} U_ac x_c;
//   transpose = 1: p_a = g_a - sum_{i in R(a)} U_ia^T p_i,
//                  l_a = D_a^-T (p_a - sum_{c > a} W_ca^T l_c).
// The parts from below the clique in one parallel pass (16 lanes per clique
// node); then the clique column by column on the first wavefront, lane a
// owning clique node a, each lane's blocks requested four columns ahead: up,
// once node b is final (after its D^-1 when transpose = 0) every node a above
// it takes node b's part; down, node c final (after its D^-T when
// transpose = 1), every node a below takes node c's part.
template <bool TRANS, bool LDSX>
__device__ void clique_solve(const DevSym& S, const View& w, double2* x2)
{
    constexpr int kAhead = 4;  // columns whose blocks are in flight
    // the part of slot (i; k) that the up sweep reads (U_ik^T or W_ki) and
    // the part of slot (a; c) the down sweep reads (W_ca^T or U_ac)
    constexpr int kUp = TRANS ? 4 : 0, kDown = TRANS ? 0 : 4;
    auto madd = [](double& y0, double& y1, const Blk& A, double x0, double x1) {
        if (TRANS) mtvadd(y0, y1, A, x0, x1);
        else mvadd(y0, y1, A, x0, x1);
    };
    const int KC = S.tail_clique, kf = S.tail_nodes - KC;
    const int64_t lu = S.lu_off;
    {
        constexpr int g = 16;
        const int grp = threadIdx.x / g, lane = threadIdx.x & (g - 1);
        for (int a0 = 0; a0 < KC; a0 += blockDim.x / g) {
            const int a = a0 + grp;
            double z0 = 0.0, z1 = 0.0;
            const int jl = kf + (a < KC ? a : 0);
            const int4 t1 = S.t_node[3 * jl + 1];
            const int rmid = S.t_node[3 * jl + 2].x;
            if (a < KC) {
                for (int r = t1.y + lane; r < t1.z; r += g) {  // outside the tail
                    const int2 e = S.t_rl[r];
                    const double2 p = x2[e.x];
                    madd(z0, z1, w.blk(lu + 8 * (int64_t)e.y + kUp), p.x, p.y);
                }
                for (int r = t1.z + lane; r < rmid; r += g) {  // the tail below the clique
                    const int2 e = S.t_rl[r];
                    const int i = S.t_node[3 * e.x].x;
                    const int sl = S.t_slot[3 * e.y].x;
                    const double2 p = x2[i];
                    madd(z0, z1, w.blk(lu + 8 * (int64_t)sl + kUp), p.x, p.y);
                }
            }
            gsum2(z0, z1, g);
            if (a < KC && lane == 0) {
                const int j = S.t_node[3 * jl].x;
                const double2 v = x2[j];
                x2[j] = make_double2(v.x - z0, v.y - z1);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < kWave) {
        const int lane = threadIdx.x;
        const bool mine = lane < KC;
        int ja = 0, lpa = 0;
        if (mine) {
            ja = S.t_node[3 * (kf + lane)].x;
            lpa = S.Lp[ja];
        }
        auto d_of = [&](int c) { return w.blk(4 * (int64_t)__shfl(ja, c)); };
        // up: the block of slot (b; lane), and (transpose = 0) D_b^-1
        auto u_of = [&](int b) {
            const int lpb = __shfl(lpa, b);
            Blk r = bzero();
            if (mine && lane > b) r = w.blk(lu + 8 * (int64_t)(lpb + lane - b - 1) + kUp);
            return r;
        };
        const int nb = TRANS ? KC - 1 : KC;  // columns of the up pass
        Blk q[kAhead], qd[kAhead];
#pragma unroll
        for (int k = 0; k < kAhead; ++k) {
            q[k] = k + 1 < KC ? u_of(k) : bzero();
            qd[k] = bzero();
            if (!TRANS && k < KC) qd[k] = d_of(k);
        }
        for (int b = 0; b < nb; ++b) {
            const Blk u = q[0], Db = qd[0];
#pragma unroll
            for (int k = 0; k + 1 < kAhead; ++k) {
                q[k] = q[k + 1];
                qd[k] = qd[k + 1];
            }
            q[kAhead - 1] = b + kAhead + 1 < KC ? u_of(b + kAhead) : bzero();
            qd[kAhead - 1] = bzero();
            if (!TRANS && b + kAhead < KC) qd[kAhead - 1] = d_of(b + kAhead);
            double2 pb = x2[__shfl(ja, b)];
            if (!TRANS) {
                double y0 = 0.0, y1 = 0.0;
                mvadd(y0, y1, Db, pb.x, pb.y);
                pb = make_double2(y0, y1);
            }
            if (mine && lane > b) {
                double z0 = 0.0, z1 = 0.0;
                madd(z0, z1, u, pb.x, pb.y);
                const double2 v = x2[ja];
                x2[ja] = make_double2(v.x - z0, v.y - z1);
            } else if (!TRANS && lane == b) {
                x2[ja] = pb;
            }
            sync_x<LDSX>();
        }
        // down: the block of slot (lane; c), and (transpose = 1) D_c^-1
        auto w_of = [&](int c) {
            Blk r = bzero();
            if (lane < c) r = w.blk(lu + 8 * (int64_t)(lpa + c - lane - 1) + kDown);
            return r;
        };
        Blk wq[kAhead], dq[kAhead];
#pragma unroll
        for (int k = 0; k < kAhead; ++k) {
            wq[k] = KC - 1 - k >= 0 ? w_of(KC - 1 - k) : bzero();
            dq[k] = bzero();
            if (TRANS && KC - 1 - k >= 0) dq[k] = d_of(KC - 1 - k);
        }
        for (int c = KC - 1; c >= 0; --c) {
            const Blk Wc = wq[0], Dc = dq[0];
#pragma unroll
            for (int k = 0; k + 1 < kAhead; ++k) {
                wq[k] = wq[k + 1];
                dq[k] = dq[k + 1];
            }
            wq[kAhead - 1] = c - kAhead >= 0 ? w_of(c - kAhead) : bzero();
            dq[kAhead - 1] = bzero();
            if (TRANS && c - kAhead >= 0) dq[kAhead - 1] = d_of(c - kAhead);
            double2 pc = x2[__shfl(ja, c)];
            if (TRANS) {
                double l0 = 0.0, l1 = 0.0;
                mtvadd(l0, l1, Dc, pc.x, pc.y);
                pc = make_double2(l0, l1);
            }
            if (lane < c) {
                double z0 = 0.0, z1 = 0.0;
                madd(z0, z1, Wc, pc.x, pc.y);
                const double2 v = x2[ja];
                x2[ja] = make_double2(v.x - z0, v.y - z1);
            } else if (TRANS && lane == c) {
                x2[ja] = pc;
            }
            sync_x<LDSX>();
        }
    }
    __syncthreads();
}

// The two sweeps of one case on the vector x2 (position order, in LDS or
// global memory), with the factors in view w; the clique chain at the top
// column by column when it fits one wavefront.
template <bool TRANS, bool LDSX>
__device__ __forceinline__ void solve_sweeps(const DevSym& S, const View& w, double2* x2)
{
    const bool col = S.tail_clique >= 3 && S.tail_clique <= kWave;
    const int L = col ? S.nlev - S.tail_clique : S.nlev;
    solve_up<TRANS>(S, w, x2, L);
    if (col) clique_solve<TRANS, LDSX>(S, w, x2);
    solve_down<TRANS>(S, w, x2, L);
}

template <bool TRANS, bool LDSX>
__global__ __launch_bounds__(kLevelThreads) void k_solve(DevSym S, const double* vals,
                                                       int64_t vals_stride, int C, int B,
                                                       double* rhs, int64_t rhs_stride)
{
    const int c = case_of_block(blockIdx.x, C, B);
    if (c < 0) return;
    const View w = case_view(const_cast<double*>(vals), vals_stride, C, c);
    double2* xg = reinterpret_cast<double2*>(rhs + c * rhs_stride);
    double2* x2 = LDSX ? reinterpret_cast<double2*>(pf_smem) : xg;
    if (LDSX) {
        for (int p = threadIdx.x; p < S.nn; p += blockDim.x) x2[p] = xg[p];
        __syncthreads();
    }
    solve_sweeps<TRANS, LDSX>(S, w, x2);
    if (LDSX) {
        __syncthreads();
        for (int p = threadIdx.x; p < S.nn; p += blockDim.x) xg[p] = x2[p];
    }
}

// Adjoint of one case with the factors of J at its solution (beyond the
// paper): the loss gradient gathered into position order,
//   g_p = (dL/dtheta, dL/d|V| or 0 at a PV bus) of bus perm[p]
// (absent gVm / gVa read as zero), the transposed solves J^T lam = g, then
// lam to the caller and the injection gradients dL/dPsp = lam_P (non-slack
// buses), dL/dQsp = lam_Q (PQ buses), 0 elsewhere.  A case whose status is
// not PF_OK (its factors are not those of a converged J) gets NaN
// gradients.
// dL/dx_e of one case from the rectangular voltages of the branch's ends and
// their adjoint entries (lam_Q already zero at PV buses); an end that is the
// slack adds nothing:
//   dS_f = V_f conj(dy (V_f - V_t)), dS_t = V_t conj(dy (V_t - V_f)),
//   dy = -j y^2, dL/dx = -(lamP_f Re dS_f + lamQ_f Im dS_f + same at t).
// Contraction into fused multiply-adds is off here, so that every kernel
// that calls this gets the same bits.
__device__ __forceinline__ double adj_branch_core(double r, double x, double ef, double ff,
                                                  double et, double ft, double lpf, double lqf,
                                                  double lpt, double lqt, bool f_in, bool t_in)
{
#pragma clang fp contract(off)
    const double den = r * r + x * x;
    const double yr = r / den, yi = -x / den;
    const double dyr = 2.0 * yr * yi, dyi = -(yr * yr - yi * yi);
    const double dr = ef - et, di = ff - ft;
    const double cr = dyr * dr - dyi * di, ci = dyr * di + dyi * dr;
    double acc = 0.0;
    if (f_in) acc += lpf * (ef * cr + ff * ci) + lqf * (ff * cr - ef * ci);
    if (t_in) acc += lpt * (-(et * cr + ft * ci)) + lqt * (-(ft * cr - et * ci));
    return -acc;
}

// The same from the bus records (e, f, lam_P, lam_Q) of the two ends.
__device__ __forceinline__ double adj_branch_rec(double r, double x, const Blk& F,
                                                 const Blk& T, bool f_in, bool t_in)
{
    return adj_branch_core(r, x, F.a, F.b, T.a, T.b, F.c, F.d, T.c, T.d, f_in, t_in);
}

template <bool LDSX>
__global__ __launch_bounds__(kLevelThreads) void k_adjoint(DevSym S, AdjArgs a)
{
    const int c = case_of_block(blockIdx.x, a.C, a.B);
    if (c < 0) return;
    const View w = case_view(const_cast<double*>(a.ws), a.ws_stride, a.C, c);
    double2* lg = reinterpret_cast<double2*>(a.lam + c * a.lam_stride);
    double2* x2 = LDSX ? reinterpret_cast<double2*>(pf_smem) : lg;
    const double* gVm = a.gVm ? a.gVm + c * a.gv_stride : nullptr;
    const double* gVa = a.gVa ? a.gVa + c * a.gv_stride : nullptr;
    const int8_t* ty = a.type + c * a.type_stride;
    for (int p = threadIdx.x; p < S.nn; p += blockDim.x) {
        const int bus = S.perm[p];
        const double ga = gVa ? gVa[bus] : 0.0;
        const double gm = (gVm && ty[bus] != T_PV) ? gVm[bus] : 0.0;
        x2[p] = make_double2(ga, gm);
    }
    __syncthreads();
    solve_sweeps<true, LDSX>(S, w, x2);
    __syncthreads();
    const bool ok = !a.status || a.status[c] == ST_OK;
    const double nan = __builtin_nan("");
    if (LDSX)
        for (int p = threadIdx.x; p < S.nn; p += blockDim.x) lg[p] = x2[p];
    double* gP = a.gP + c * a.g_stride;
    double* gQ = a.gQ + c * a.g_stride;
    for (int i = threadIdx.x; i < S.n; i += blockDim.x) {
        const int p = S.pos[i];
        double lp = 0.0, lq = 0.0;
        if (p >= 0) {
            const double2 l = x2[p];
            lp = l.x;
            lq = ty[i] == T_PV ? 0.0 : l.y;
        }
        gP[i] = ok ? lp : nan;
        gQ[i] = ok ? lq : nan;
    }
    if (a.gx_mode < 0) return;
    // dL/dx of this case's branches: per bus (e, f, lam_P, lam_Q) into the
    // first half of its workspace bus record (the masks of the gradients
    // above applied), then per branch the two records; with gx_mode 1 each
    // case's values go to the workspace's rhs section for k_adj_gx_sum
    const View wb = case_bus_view(a.ws, a.ws_stride, a.C, c, S.vals_doubles);
    const Off o = ws_off(S);
    const double* Vm = a.Vm + c * a.v_stride;
    const double* Va = a.Va + c * a.v_stride;
    for (int i = threadIdx.x; i < S.n; i += blockDim.x) {
        double sn, cs;
        sincos(Va[i], &sn, &cs);
        const int p = S.pos[i];
        double lp = 0.0, lq = 0.0;
        if (p >= 0) {
            const double2 l = x2[p];
            lp = l.x;
            lq = ty[i] == T_PV ? 0.0 : l.y;
        }
        wb.put(o.BUS + 8 * (int64_t)i, {Vm[i] * cs, Vm[i] * sn, lp, lq});
    }
    __syncthreads();
    const double* r = a.r + c * a.branch_stride;
    const double* x = a.x + c * a.branch_stride;
    for (int e = threadIdx.x; e < S.m; e += blockDim.x) {
        const int fb = a.from[e], tb = a.to[e];
        const Blk F = wb.blk(o.BUS + 8 * (int64_t)fb);
        const Blk T = wb.blk(o.BUS + 8 * (int64_t)tb);
        const double v = ok ? adj_branch_rec(r[e], x[e], F, T, fb != S.slack, tb != S.slack)
                            : nan;
        if (a.gx_mode == 0) a.gx[(int64_t)c * S.m + e] = v;
        else *wb.at(o.RHS + e) = v;
    }
}

template <bool MULTI>
__global__ __launch_bounds__(kLevelThreads) void k_newton(DevSym Sarg,
                                                        const CaseDesc* __restrict__ descs,
                                                        const int32_t* __restrict__ order,
                                                        NewtonArgs a)
{
    if (MULTI) {
        const int c = order[blockIdx.x];
        const CaseDesc& cd = descs[c];
        const DevSym S = cd.sym;
        const View w = case_view(a.ws + cd.ws_off, 0, 1, 0);
        const View wb = case_bus_view(a.ws + cd.ws_off, 0, 1, 0, S.vals_doubles);
        newton_case(OneGroup{}, S, a.yval + cd.y_off, a.type + cd.bus_off, a.Psp + cd.bus_off,
                    a.Qsp + cd.bus_off, a.Vm + cd.bus_off, a.Va + cd.bus_off, w, wb, a.tol,
                    a.max_iter, a.flags, a.iters ? a.iters + c : nullptr,
                    a.norm ? a.norm + c : nullptr, a.status ? a.status + c : nullptr,
                    a.pivot ? a.pivot + c : nullptr);
    } else {
        const int c = case_of_block(blockIdx.x, a.interleave, a.B);
        if (c < 0) return;
        const View w = case_view(a.ws, a.ws_stride, a.interleave, c);
        const View wb = case_bus_view(a.ws, a.ws_stride, a.interleave, c, Sarg.vals_doubles);
        newton_case(OneGroup{}, Sarg, a.yval + c * a.y_stride, a.type + c * a.type_stride,
                    a.Psp + c * a.inj_stride, a.Qsp + c * a.inj_stride, a.Vm + c * a.v_stride,
                    a.Va + c * a.v_stride, w, wb, a.tol, a.max_iter, a.flags,
                    a.iters ? a.iters + c : nullptr, a.norm ? a.norm + c : nullptr,
                    a.status ? a.status + c : nullptr, a.pivot ? a.pivot + c : nullptr);
    }
}

// One case over every workgroup of a cooperative launch; sync: the case's
// grid-barrier words (three 128-byte lines, see Spread).
__global__ __launch_bounds__(kLevelThreads) void k_newton_spread(DevSym S, NewtonArgs a,
                                                               unsigned* sync, int back_lo,
                                                               unsigned long long wait_ticks)
{
    __shared__ unsigned s_count;
    if (threadIdx.x == 0) s_count = 0;
    const Spread par{sync,    sync + 32,          reinterpret_cast<int*>(sync + 64),
                     reinterpret_cast<uint64_t*>(sync + 68), &s_count, back_lo, wait_ticks,
                     (int)blockIdx.x, (int)gridDim.x};
    const View w = case_view(a.ws, a.ws_stride, 1, 0);
    const View wb = case_bus_view(a.ws, a.ws_stride, 1, 0, S.vals_doubles);
    newton_case(par, S, a.yval, a.type, a.Psp, a.Qsp, a.Vm, a.Va, w, wb, a.tol, a.max_iter,
                a.flags, a.iters, a.norm, a.status, a.pivot);
}

// A batch of grids (each case its own symbolic) in one cooperative launch
// with more workgroups than cases: blocks[b] = (case, rank, group size) of
// workgroup b.  A case with one workgroup runs as in k_newton<true>; a
// larger group shares its case as a spread launch does, with grid barriers
// among the group's workgroups only.
__global__ __launch_bounds__(kLevelThreads) void k_newton_multi_spread(
    const CaseDesc* __restrict__ descs, const int4* __restrict__ blocks, NewtonArgs a,
    unsigned long long wait_ticks)
{
    __shared__ unsigned s_count;
    const int4 bk = blocks[blockIdx.x];
    const int c = bk.x;
    const CaseDesc& cd = descs[c];
    const DevSym S = cd.sym;
    const View w = case_view(a.ws + cd.ws_off, 0, 1, 0);
    const View wb = case_bus_view(a.ws + cd.ws_off, 0, 1, 0, S.vals_doubles);
    const double* yv = a.yval + cd.y_off;
    const int8_t* ty = a.type + cd.bus_off;
    const double* P = a.Psp + cd.bus_off;
    const double* Q = a.Qsp + cd.bus_off;
    double* Vm = a.Vm + cd.bus_off;
    double* Va = a.Va + cd.bus_off;
    int32_t* o_it = a.iters ? a.iters + c : nullptr;
    double* o_nrm = a.norm ? a.norm + c : nullptr;
    int32_t* o_st = a.status ? a.status + c : nullptr;
    int32_t* o_pv = a.pivot ? a.pivot + c : nullptr;
    if (bk.z <= 1) {
        newton_case(OneGroup{}, S, yv, ty, P, Q, Vm, Va, w, wb, a.tol, a.max_iter, a.flags, o_it,
                    o_nrm, o_st, o_pv);
        return;
    }
    if (threadIdx.x == 0) s_count = 0;
    unsigned* sync = reinterpret_cast<unsigned*>(a.ws + cd.ws_off + cd.sync_off);
    const SpreadSub par{{sync, sync + 32, reinterpret_cast<int*>(sync + 64),
                         reinterpret_cast<uint64_t*>(sync + 68), &s_count, cd.back_lo,
                         wait_ticks, bk.y, bk.z}};
    newton_case(par, S, yv, ty, P, Q, Vm, Va, w, wb, a.tol, a.max_iter, a.flags, o_it, o_nrm,
                o_st, o_pv);
}

// Clears the grid-barrier words before a spread launch (a kernel, not a
// memset, so that the pair can be recorded into a graph); the pivot marker
// starts at kNoPivot.
__global__ void k_spread_init(unsigned* sync)
{
    const int i = threadIdx.x;
    if (i < kSpreadWords) sync[i] = i == 65 ? (unsigned)kNoPivot : 0u;
}

// The same for every case of a batch of grids whose group has more than one
// workgroup (block c: case c).
__global__ void k_spread_init_multi(const CaseDesc* __restrict__ descs, double* ws)
{
    const CaseDesc& cd = descs[blockIdx.x];
    if (cd.spread <= 1) return;
    unsigned* sync = reinterpret_cast<unsigned*>(ws + cd.ws_off + cd.sync_off);
    const int i = threadIdx.x;
    if (i < kSpreadWords) sync[i] = i == 65 ? (unsigned)kNoPivot : 0u;
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

// dL/dx_e for one case from the case's |V|, theta and adjoint vector (by
// position); the arithmetic of adj_branch_core.
__device__ __forceinline__ double adj_branch(const DevSym& S, int fb, int tb,
                                             const double* lam, const int8_t* type,
                                             const double* Vm, const double* Va, double r,
                                             double x)
{
    double sf, cf, st, ct;
    sincos(Va[fb], &sf, &cf);
    sincos(Va[tb], &st, &ct);
    const int pf_ = S.pos[fb], pt_ = S.pos[tb];
    const double2* l2 = reinterpret_cast<const double2*>(lam);
    double lpf = 0.0, lqf = 0.0, lpt = 0.0, lqt = 0.0;
    if (pf_ >= 0) {
        const double2 l = l2[pf_];
        lpf = l.x;
        lqf = (type[fb] == T_PV) ? 0.0 : l.y;
    }
    if (pt_ >= 0) {
        const double2 l = l2[pt_];
        lpt = l.x;
        lqt = (type[tb] == T_PV) ? 0.0 : l.y;
    }
    return adj_branch_core(r, x, Vm[fb] * cf, Vm[fb] * sf, Vm[tb] * ct, Vm[tb] * st, lpf, lqf,
                           lpt, lqt, pf_ >= 0, pt_ >= 0);
}

// dL/dx summed over the cases from the per-case values k_adjoint left in
// each case's rhs section of the workspace, in the order of k_adj_branch's
// mode 1 (wave w sums the cases w, w + 16, ..., then the 16 partial sums in
// wave order), so both give the same bits.
__global__ void k_adj_gx_sum(DevSym S, const double* ws, int64_t ws_stride, int C, int B,
                             double* gx)
{
    __shared__ double part[16][64];
    const int e = blockIdx.x * 64 + (threadIdx.x & 63);
    const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const Off o = ws_off(S);
    double acc = 0.0;
    if (e < S.m)
        for (int c = wv; c < B; c += nw)
            acc += *case_bus_view(const_cast<double*>(ws), ws_stride, C, c, S.vals_doubles)
                        .at(o.RHS + e);
    part[wv][threadIdx.x & 63] = acc;
    __syncthreads();
    if (wv == 0 && e < S.m) {
        double sum = 0.0;
        for (int k = 0; k < nw; ++k) sum += part[k][threadIdx.x];
        gx[e] = sum;
    }
}

// mode 1 (x shared by the cases): one workgroup per 64 branches, its waves
// split the cases and combine them in a fixed order, so no atomics are
// needed and the sum is reproducible.  mode 0: one thread per (case, branch).
// A case whose status (if given) is not PF_OK contributes NaN.
__global__ void k_adj_branch(DevSym S, const int32_t* __restrict__ from,
                             const int32_t* __restrict__ to, int B, const double* lam,
                             int64_t lam_stride, const int8_t* type, int64_t type_stride,
                             const double* Vm, const double* Va, int64_t v_stride,
                             const double* r, const double* x, int64_t branch_stride,
                             const int32_t* status, double* gx, int mode)
{
    const double nan = __builtin_nan("");
    if (mode == 1) {
        __shared__ double part[16][64];
        const int e = blockIdx.x * 64 + (threadIdx.x & 63);
        const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
        double acc = 0.0;
        if (e < S.m) {
            const int fb = from[e], tb = to[e];
            for (int c = wv; c < B; c += nw)
                acc += (status && status[c] != ST_OK)
                           ? nan
                           : adj_branch(S, fb, tb, lam + c * lam_stride, type + c * type_stride,
                                        Vm + c * v_stride, Va + c * v_stride,
                                        r[c * branch_stride + e], x[c * branch_stride + e]);
        }
        part[wv][threadIdx.x & 63] = acc;
        __syncthreads();
        if (wv == 0 && e < S.m) {
            double s = 0.0;
            for (int k = 0; k < nw; ++k) s += part[k][threadIdx.x];
            gx[e] = s;
        }
    } else {
        const int e = blockIdx.x * blockDim.x + threadIdx.x;
        const int c = blockIdx.y;
        if (e >= S.m) return;
        gx[(int64_t)c * S.m + e] =
            (status && status[c] != ST_OK)
                ? nan
                : adj_branch(S, from[e], to[e], lam + c * lam_stride, type + c * type_stride,
                             Vm + c * v_stride, Va + c * v_stride, r[c * branch_stride + e],
                             x[c * branch_stride + e]);
    }
}


struct pf_multi_s {

    std::vector<pf_symbolic> syms;
    std::vector<int64_t> bus_off, br_off, y_off, ws_off;
    std::vector<int64_t> work;   // estimated one-workgroup work of each case
    std::vector<int32_t> order;  // cases by decreasing work
    std::vector<uint64_t> gens;  // each symbolic's upload count when the plan was uploaded
    // workgroups of pf_newton_multi's launch (0: one per case) and their
    // assignment: counts[c] workgroups for case c; blocks: (case, rank,
    // group size, 0) per workgroup
    int spread = 0;
    std::vector<int32_t> counts;
    std::vector<int32_t> blocks;
    const CaseDesc* d_desc = nullptr;
    const int32_t* d_order = nullptr;
    const int4* d_blocks = nullptr;
    bool uploaded = false;
};


namespace {

// Dynamic LDS of the Newton kernel: the tail and the (e, f) copy share the
// front, the PV mask follows the larger of the two.
int newton_lds(const HostSym& h)
{
    return std::max(h.tail_lds, h.ef_lds) + (int)pv_mask_bytes(h.n);
}

// Raises the dynamic-LDS limit of the level-scheduled kernels to what the
// device allows (160 KB per workgroup on gfx950) minus their static LDS.
// Failures only keep the default limit; the sticky error is cleared so that
// it is not reported by the next launch check.
void allow_big_lds()
{
    static bool done = false;
    if (done) return;
    done = true;
    int dev = 0, lds_max = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
            hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    const void* kernels[] = {reinterpret_cast<const void*>(&k_adjoint<true>),
                             reinterpret_cast<const void*>(&k_newton<false>),
                             reinterpret_cast<const void*>(&k_newton<true>),
                             reinterpret_cast<const void*>(&k_newton_spread),
                             reinterpret_cast<const void*>(&k_newton_multi_spread),
                             reinterpret_cast<const void*>(&k_factor<false>),
                             reinterpret_cast<const void*>(&k_factor<true>),
                             reinterpret_cast<const void*>(&k_solve<false, true>),
                             reinterpret_cast<const void*>(&k_solve<true, true>)};
    for (const void* k : kernels) {
        hipFuncAttributes fa{};
        if (hipFuncGetAttributes(&fa, k) == hipSuccess) {
            const int dyn = lds_max - (int)fa.sharedSizeBytes;
            if (dyn > 0)
                (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
        }
    }
    (void)hipGetLastError();
}

// Workgroups of a one-case Newton launch spread over the device: the
// symbolic's setting, capped by the workgroups the device keeps resident at
// once (a cooperative launch needs every one of them at the same time); 0
// selects the one-workgroup kernel, which also serves batches and every
// launch recorded into a graph.
int spread_blocks(const HostSym& h, int B, int threads, int lds, hipStream_t st)
{
    if (B != 1 || h.spread <= 1) return 0;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    int dev = 0, cus = 0, per = 0;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_newton_spread, threads, lds) !=
            hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    const int G = std::min(h.spread, per * cus);
    return G > 1 ? G : 0;
}

// The Newton launch of pf_newton and pf_newton_noalloc (arguments checked).
int newton_launch(const HostSym& h, int B, int C, NewtonArgs a, hipStream_t st, const char* fn)
{
    allow_big_lds();
    const int threads = launch_threads(h, B);
    const int lds = newton_lds(h);
    const int G = spread_blocks(h, B, threads, lds, st);
    if (G > 1) {
        unsigned* sync = reinterpret_cast<unsigned*>(a.ws + h.sync_off());
        hipLaunchKernelGGL(k_spread_init, dim3(1), dim3(128), 0, st, sync);
        if (const int e = launch_check(fn)) return e;
        DevSym S = h.dev;
        // the narrow global levels (at most one node per thread of a
        // workgroup) go with the tail's backward substitution
        int back_lo = h.tail_level;
        while (back_lo > 0 && h.level_ptr[back_lo] - h.level_ptr[back_lo - 1] <= threads)
            --back_lo;
        unsigned long long wait = h.spread_wait;
        void* args[] = {&S, &a, &sync, &back_lo, &wait};
        return hip_check(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_newton_spread),
                                                    dim3(G), dim3(threads), args,
                                                    (unsigned)lds, st),
                         fn);
    }
    hipLaunchKernelGGL(k_newton<false>, dim3(grid_blocks(B, C)), dim3(threads), lds, st, h.dev,
                       (const CaseDesc*)nullptr, (const int32_t*)nullptr, a);
    return launch_check(fn);
}

// Threads per workgroup of pf_newton_multi's launch: the largest setting of
// the plan's symbolics, else 512 up to 512 cases and 256 beyond.
int multi_threads(const pf_multi p)
{
    int threads = 0;
    for (auto* sy : p->syms) threads = std::max(threads, sy->h.threads);
    if (threads == 0) threads = (p->syms.size() <= 512) ? 512 : 256;
    return threads;
}

// First level of the backward sweep left to a spread group's first
// workgroup: the narrow global levels (at most one node per thread).
int spread_back_lo(const HostSym& h, int threads)
{
    int lo = h.tail_level;
    while (lo > 0 && h.level_ptr[lo] - h.level_ptr[lo - 1] <= threads) --lo;
    return lo;
}

// Workgroups per case for a launch of `spread` workgroups in all: one each,
// then the rest one at a time to the case with the most work per workgroup
// (each case at most one per 128 nodes of its widest level below the tail,
// and 32), so that the largest grids, which bound the launch, share theirs.
void plan_blocks(pf_multi p)
{
    const int G = (int)p->syms.size();
    p->counts.assign(G, 1);
    std::vector<int> cap(G, 1);
    for (int c = 0; c < G; ++c) {
        const HostSym& h = p->syms[c]->h;
        int widest = 0;
        for (int l = 0; l < h.tail_level; ++l)
            widest = std::max(widest, h.level_ptr[l + 1] - h.level_ptr[l]);
        cap[c] = std::max(1, std::min(32, widest / 128));
    }
    int extra = std::max(0, p->spread - G);
    while (extra > 0) {
        int best = -1;
        for (int c = 0; c < G; ++c) {
            if (p->counts[c] >= cap[c]) continue;
            // work per workgroup, compared without division
            if (best < 0 || p->work[c] * p->counts[best] > p->work[best] * p->counts[c]) best = c;
        }
        if (best < 0) break;
        ++p->counts[best];
        --extra;
    }
    p->blocks.clear();
    for (int c : p->order)
        for (int r = 0; r < p->counts[c]; ++r) {
            p->blocks.push_back(c);
            p->blocks.push_back(r);
            p->blocks.push_back(p->counts[c]);
            p->blocks.push_back(0);
        }
}

}  // namespace

namespace pf {
namespace abi {

// The level-scheduled factorisation of B matrices (sym: symmetric ones).
void factor_launch(const HostSym& h, int B, double* vals, int64_t stride, int C,
                   int32_t* status, int32_t* pivot, hipStream_t st, bool sym)
{
    allow_big_lds();
    if (sym)
        hipLaunchKernelGGL(k_factor<true>, dim3(grid_blocks(B, C)), dim3(launch_threads(h, B)),
                           h.tail_lds, st, h.dev, vals, stride, C, B, status, pivot);
    else
        hipLaunchKernelGGL(k_factor<false>, dim3(grid_blocks(B, C)), dim3(launch_threads(h, B)),
                           h.tail_lds, st, h.dev, vals, stride, C, B, status, pivot);
}

}  // namespace abi
}  // namespace pf

extern "C" {
int pf_build_ybus(const pf_symbolic s, int B, const double* d_r, const double* d_x,
                  const double* d_b, int64_t branch_stride, const double* d_ysh,
                  int64_t ysh_stride, double* d_yval, int64_t y_stride, void* stream)
{
    if (!ready(s, "pf_build_ybus")) return PF_E_INVALID;
    if (B < 0 || B > 65535 || !d_r || !d_x || !d_b || !d_yval || branch_stride < 0 ||
        ysh_stride < 0)
        return fail(PF_E_INVALID, "pf_build_ybus: bad arguments");
    if (B > 1 && y_stride < 2 * (int64_t)s->h.ycol.size())
        return fail(PF_E_WORKSPACE, "pf_build_ybus: y_stride < 2*nnz_y");
    if (B > 1 && branch_stride != 0 && branch_stride < s->h.m)
        return fail(PF_E_WORKSPACE, "pf_build_ybus: branch_stride < m");
    if (d_ysh && ((ysh_stride & 1) || (B > 1 && ysh_stride != 0 && ysh_stride < 2 * s->h.n) ||
                  (reinterpret_cast<uintptr_t>(d_ysh) & 15)))
        return fail(PF_E_INVALID, "pf_build_ybus: ysh_stride must be 0 or even and >= 2*n, "
                                  "d_ysh 16-byte aligned");
    if (B == 0) return PF_OK;
    dim3 grid((unsigned)(((int64_t)s->h.n * kYbusLanes + 255) / 256), B);
    hipLaunchKernelGGL(k_ybus, grid, dim3(256), 0, as_stream(stream), s->h.dev, d_r, d_x, d_b,
                       branch_stride, d_ysh, ysh_stride, d_yval, y_stride);
    return launch_check("pf_build_ybus");
}

int pf_mismatch(const pf_symbolic s, int B, const double* d_yval, int64_t y_stride,
                const int8_t* d_type, int64_t type_stride, const double* d_Psp,
                const double* d_Qsp, int64_t inj_stride, const double* d_Vm, const double* d_Va,
                int64_t v_stride, double* d_rhs, int64_t rhs_stride, double* d_norm,
                double* d_PQ, void* stream)
{
    if (!ready(s, "pf_mismatch")) return PF_E_INVALID;
    if (B < 0 || !d_yval || !d_type || !d_Psp || !d_Qsp || !d_Vm || !d_Va || !d_rhs ||
        v_stride < 0 || rhs_stride < 0)
        return fail(PF_E_INVALID, "pf_mismatch: bad arguments");
    if (!shared_stride_ok(B, y_stride, 2 * (int64_t)s->h.ycol.size()) ||
        !shared_stride_ok(B, type_stride, s->h.n) || !shared_stride_ok(B, inj_stride, s->h.n) ||
        (B > 1 && (v_stride < s->h.n || rhs_stride < 2 * (int64_t)s->h.nn)))
        return fail(PF_E_WORKSPACE, "pf_mismatch: a stride is too small or negative");
    if (B == 0) return PF_OK;
    hipLaunchKernelGGL(k_mismatch, dim3(B), dim3(256), 0, as_stream(stream), s->h.dev, d_yval,
                       y_stride, d_type, type_stride, d_Psp, d_Qsp, inj_stride, d_Vm, d_Va,
                       v_stride, d_rhs, rhs_stride, d_norm, d_PQ);
    return launch_check("pf_mismatch");
}

int pf_jacobian(const pf_symbolic s, int B, const double* d_yval, int64_t y_stride,
                const int8_t* d_type, int64_t type_stride, const double* d_Vm, const double* d_Va,
                int64_t v_stride, double* d_vals, int64_t vals_stride, int vals_interleave,
                void* stream)
{
    if (!ready(s, "pf_jacobian")) return PF_E_INVALID;
    if (B < 0 || B > 65535 || !d_yval || !d_type || !d_Vm || !d_Va || !d_vals ||
        !valid_interleave(vals_interleave) || (vals_stride & 7))
        return fail(PF_E_INVALID, "pf_jacobian: bad arguments");
    if (B > 1 && vals_stride < s->h.vals_doubles())
        return fail(PF_E_WORKSPACE, "pf_jacobian: vals_stride < vals_doubles");
    if (!shared_stride_ok(B, y_stride, 2 * (int64_t)s->h.ycol.size()) ||
        !shared_stride_ok(B, type_stride, s->h.n) || v_stride < 0 ||
        (B > 1 && v_stride < s->h.n))
        return fail(PF_E_WORKSPACE, "pf_jacobian: a stride is too small or negative");
    if (B == 0 || s->h.nn == 0) return PF_OK;
    dim3 grid((s->h.nn + 255) / 256, B);
    hipLaunchKernelGGL(k_jacobian, grid, dim3(256), 0, as_stream(stream), s->h.dev, d_yval,
                       y_stride, d_type, type_stride, d_Vm, d_Va, v_stride, d_vals, vals_stride,
                       vals_interleave);
    return launch_check("pf_jacobian");
}

int pf_factor(const pf_symbolic s, int B, double* d_vals, int64_t vals_stride,
              int vals_interleave, int32_t* d_status, int32_t* d_pivot, void* stream)
{
    if (!ready(s, "pf_factor")) return PF_E_INVALID;
    if (B < 0 || !d_vals || !valid_interleave(vals_interleave) || (vals_stride & 7))
        return fail(PF_E_INVALID, "pf_factor: bad arguments");
    if (B > 1 && vals_stride < s->h.vals_doubles())
        return fail(PF_E_WORKSPACE, "pf_factor: vals_stride < vals_doubles");
    if (B == 0) return PF_OK;
    factor_launch(s->h, B, d_vals, vals_stride, vals_interleave, d_status, d_pivot,
                  as_stream(stream), false);
    return launch_check("pf_factor");
}

int pf_solve(const pf_symbolic s, int B, const double* d_vals, int64_t vals_stride,
             int vals_interleave, double* d_rhs, int64_t rhs_stride, int transpose, void* stream)
{
    if (!ready(s, "pf_solve")) return PF_E_INVALID;
    if (B < 0 || !d_vals || !d_rhs || (transpose != 0 && transpose != 1) ||
        !valid_interleave(vals_interleave) || (vals_stride & 7))
        return fail(PF_E_INVALID, "pf_solve: bad arguments");
    if (B > 1 && rhs_stride < 2 * (int64_t)s->h.nn)
        return fail(PF_E_WORKSPACE, "pf_solve: rhs_stride < 2*nn");
    if (B == 0) return PF_OK;
    const dim3 grid(grid_blocks(B, vals_interleave)), block(launch_threads(s->h, B));
    // the case's vector in LDS when it fits beside nothing else (nn x 16 bytes)
    const size_t xbytes = 16 * (size_t)s->h.nn;
    const bool lds = xbytes <= kSolveLdsMax;
    if (lds) allow_big_lds();
    auto go = [&](auto kern, size_t shm) {
        hipLaunchKernelGGL(kern, grid, block, shm, as_stream(stream), s->h.dev, d_vals,
                           vals_stride, vals_interleave, B, d_rhs, rhs_stride);
    };
    if (transpose) {
        if (lds) go(k_solve<true, true>, xbytes);
        else go(k_solve<true, false>, 0);
    } else {
        if (lds) go(k_solve<false, true>, xbytes);
        else go(k_solve<false, false>, 0);
    }
    return launch_check("pf_solve");
}

}  // extern "C"

// ---- the allocation-free Newton entry point -------------------------------
// The Newton workspace of pf_newton_noalloc lives in this file-scope device
// array (each GPU holds its own copy for the life of the process).  Host code
// never passes the array's name to a kernel: its device address, taken once
// per device with hipGetSymbolAddress, is what the launch receives.
namespace {
constexpr int64_t kScratchDoubles = PF_NOALLOC_SCRATCH_BYTES / 8;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array, or null (with the
// error recorded) when it cannot be taken.
double* scratch_ptr(const char* fn)
{
    int dev = 0;
    if (hip_check(hipGetDevice(&dev), fn)) return nullptr;
    if (dev < 0 || dev >= kMaxDevices) {
        fail(PF_E_HIP, std::string(fn) + ": device index out of range");
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), fn)) return nullptr;
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    return g_scratch_ptr[dev];
}
}  // namespace

extern "C" {

int pf_newton_noalloc(const pf_symbolic s, int B, const double* d_yval, int64_t y_stride,
                      const int8_t* d_type, int64_t type_stride, const double* d_Psp,
                      const double* d_Qsp, int64_t inj_stride, double* d_Vm, double* d_Va,
                      int64_t v_stride, double tol, int max_iter, int32_t* d_iters,
                      double* d_norm, int32_t* d_status, int32_t* d_pivot, void* stream)
{
    if (!ready(s, "pf_newton_noalloc")) return PF_E_INVALID;
    if (B < 0 || B > 65535 || max_iter < 0 || !(tol >= 0.0) || !d_yval || !d_type || !d_Psp ||
        !d_Qsp || !d_Vm || !d_Va)
        return fail(PF_E_INVALID, "pf_newton_noalloc: bad arguments");
    if (B > 1 && v_stride < s->h.n)
        return fail(PF_E_WORKSPACE, "pf_newton_noalloc: v_stride too small");
    if (!shared_stride_ok(B, y_stride, 2 * (int64_t)s->h.ycol.size()) ||
        !shared_stride_ok(B, type_stride, s->h.n) || !shared_stride_ok(B, inj_stride, s->h.n))
        return fail(PF_E_WORKSPACE, "pf_newton_noalloc: a stride is too small or negative");
    if (B == 0) return PF_OK;
    const int C = newton_interleave(s->h, B);
    const int64_t ws_stride = s->h.ws_doubles();
    // workspace rows of whole interleaved groups (the padding blocks of the
    // grid own no case and touch no workspace)
    const int64_t need = (int64_t)((B + C - 1) / C) * C * ws_stride;
    if (need > kScratchDoubles)
        return fail(PF_E_WORKSPACE,
                    "pf_newton_noalloc: the batch needs " + std::to_string(need * 8) +
                        " bytes of workspace, more than the " +
                        std::to_string(PF_NOALLOC_SCRATCH_BYTES) +
                        "-byte scratch array; split the batch or use pf_newton");
    double* ws = scratch_ptr("pf_newton_noalloc");
    if (!ws) return PF_E_HIP;
    NewtonArgs a{d_yval, y_stride, d_type, type_stride, d_Psp, d_Qsp, inj_stride, d_Vm, d_Va,
                 v_stride, ws, ws_stride, tol, max_iter, 0, C, B, d_iters, d_norm, d_status,
                 d_pivot};
    return newton_launch(s->h, B, C, a, as_stream(stream), "pf_newton_noalloc");
}

int pf_newton(const pf_symbolic s, int B, const double* d_yval, int64_t y_stride,
              const int8_t* d_type, int64_t type_stride, const double* d_Psp,
              const double* d_Qsp, int64_t inj_stride, double* d_Vm, double* d_Va,
              int64_t v_stride, double tol, int max_iter, int flags, double* d_ws,
              int64_t ws_stride, int32_t* d_iters, double* d_norm, int32_t* d_status,
              int32_t* d_pivot, void* stream)
{
    if (!ready(s, "pf_newton")) return PF_E_INVALID;
    if (B < 0 || max_iter < 0 || !(tol >= 0.0) || !d_yval || !d_type || !d_Psp || !d_Qsp ||
        !d_Vm || !d_Va || !d_ws)
        return fail(PF_E_INVALID, "pf_newton: bad arguments");
    if (B > 1 && v_stride < s->h.n)
        return fail(PF_E_WORKSPACE, "pf_newton: v_stride too small");
    if (!shared_stride_ok(B, y_stride, 2 * (int64_t)s->h.ycol.size()) ||
        !shared_stride_ok(B, type_stride, s->h.n) || !shared_stride_ok(B, inj_stride, s->h.n))
        return fail(PF_E_WORKSPACE, "pf_newton: a stride is too small or negative");
    if (ws_stride < s->h.ws_doubles() || (ws_stride & 7))
        return fail(PF_E_WORKSPACE, "pf_newton: ws_stride must be >= ws_doubles, a multiple of 8");
    if (reinterpret_cast<uintptr_t>(d_ws) & 15)
        return fail(PF_E_WORKSPACE, "pf_newton: workspace must be 16-byte aligned");
    if (B == 0) return PF_OK;
    const int C = newton_interleave(s->h, B);
    NewtonArgs a{d_yval, y_stride, d_type, type_stride, d_Psp, d_Qsp, inj_stride, d_Vm, d_Va,
                 v_stride, d_ws, ws_stride, tol, max_iter, flags, C, B, d_iters, d_norm,
                 d_status, d_pivot};
    return newton_launch(s->h, B, C, a, as_stream(stream), "pf_newton");
}

int pf_adjoint_params(const pf_symbolic s, int B, const double* d_lam, int64_t lam_stride,
                      const int8_t* d_type, int64_t type_stride, const double* d_Vm,
                      const double* d_Va, int64_t v_stride, const double* d_r,
                      const double* d_x, int64_t branch_stride, double* d_gP, double* d_gQ,
                      int64_t g_stride, double* d_gx, int gx_mode, void* stream)
{
    return pf::abi::adjoint_branch_launch(s, B, d_lam, lam_stride, d_type, type_stride, d_Vm,
                                          d_Va, v_stride, d_r, d_x, branch_stride, nullptr,
                                          d_gP, d_gQ, g_stride, d_gx, gx_mode, stream, true);
}

int pf_adjoint(const pf_symbolic s, int B, double* d_ws, int64_t ws_stride,
               const double* d_gVm, const double* d_gVa, int64_t gv_stride, const int8_t* d_type,
               int64_t type_stride, const double* d_Vm, const double* d_Va, int64_t v_stride,
               const double* d_r, const double* d_x, int64_t branch_stride,
               const int32_t* d_status, double* d_lam, int64_t lam_stride, double* d_gP,
               double* d_gQ, int64_t g_stride, double* d_gx, int gx_mode, void* stream)
{
    if (!ready(s, "pf_adjoint")) return PF_E_INVALID;
    if (B < 0 || B > 65535 || !d_ws || !d_type || !d_Vm || !d_Va || !d_lam || !d_gP || !d_gQ ||
        (gx_mode != 0 && gx_mode != 1) || (ws_stride & 7) || gv_stride < 0 || v_stride < 0 ||
        g_stride < 0 || lam_stride < 0 || branch_stride < 0 || type_stride < 0)
        return fail(PF_E_INVALID, "pf_adjoint: bad arguments");
    if (ws_stride < s->h.ws_doubles())
        return fail(PF_E_WORKSPACE, "pf_adjoint: ws_stride < ws_doubles");
    if (B > 1 && (lam_stride < 2 * (int64_t)s->h.nn || g_stride < s->h.n ||
                  v_stride < s->h.n || (gv_stride != 0 && gv_stride < s->h.n) ||
                  (type_stride != 0 && type_stride < s->h.n) ||
                  (branch_stride != 0 && branch_stride < s->h.m)))
        return fail(PF_E_WORKSPACE, "pf_adjoint: a stride is too small");
    if (B == 0) return PF_OK;
    const int C = newton_interleave(s->h, B);
    // the branch gradients run in the adjoint launch (their per-case values
    // summed by k_adj_gx_sum for a shared x) when the workspace's rhs section
    // holds a case's m values; otherwise in their own kernel afterwards
    const HostSym& h = s->h;
    const bool fuse = d_gx && h.m > 0 && (gx_mode == 0 || h.m <= 2 * (int64_t)h.nn);
    if (d_gx && h.m > 0 && (!d_r || !d_x)) return fail(PF_E_INVALID, "pf_adjoint: need r and x");
    AdjArgs a{d_ws, ws_stride, C, B, d_gVm, d_gVa, gv_stride, d_type, type_stride, d_status,
              d_lam, lam_stride, d_gP, d_gQ, g_stride, s->d_from, s->d_to, d_Vm, d_Va, v_stride,
              d_r, d_x, branch_stride, gx_mode == 0 ? d_gx : nullptr, fuse ? gx_mode : -1};
    const size_t xbytes = 16 * (size_t)h.nn;
    const dim3 grid(grid_blocks(B, C)), block(launch_threads(h, B));
    if (xbytes <= kSolveLdsMax) {
        allow_big_lds();
        hipLaunchKernelGGL(k_adjoint<true>, grid, block, xbytes, as_stream(stream), h.dev, a);
    } else {
        hipLaunchKernelGGL(k_adjoint<false>, grid, block, 0, as_stream(stream), h.dev, a);
    }
    int rc = launch_check("pf_adjoint");
    if (rc) return rc;
    if (fuse) {
        if (gx_mode == 0) return PF_OK;
        hipLaunchKernelGGL(k_adj_gx_sum, dim3((h.m + 63) / 64), dim3(1024), 0, as_stream(stream),
                           h.dev, d_ws, ws_stride, C, B, d_gx);
        return launch_check("pf_adjoint");
    }
    return pf::abi::adjoint_branch_launch(s, B, d_lam, lam_stride, d_type, type_stride, d_Vm,
                                          d_Va, v_stride, d_r, d_x, branch_stride, d_status,
                                          nullptr, nullptr, 0, d_gx, gx_mode, stream, false);
}

}  // extern "C"

namespace pf {
namespace abi {
// Branch gradients (and, with bus, the injection gradients) of B cases from
// their adjoint vectors.
int adjoint_branch_launch(const pf_symbolic s, int B, const double* d_lam, int64_t lam_stride,
                          const int8_t* d_type, int64_t type_stride, const double* d_Vm,
                          const double* d_Va, int64_t v_stride, const double* d_r,
                          const double* d_x, int64_t branch_stride, const int32_t* d_status,
                          double* d_gP, double* d_gQ, int64_t g_stride, double* d_gx,
                          int gx_mode, void* stream, bool bus)
{
    if (!ready(s, "pf_adjoint_params")) return PF_E_INVALID;
    if (B < 0 || B > 65535 || !d_lam || !d_type || !d_Vm || !d_Va ||
        (gx_mode != 0 && gx_mode != 1) || lam_stride < 0 || type_stride < 0 || v_stride < 0 ||
        branch_stride < 0 || g_stride < 0)
        return fail(PF_E_INVALID, "pf_adjoint_params: bad arguments");
    const HostSym& h = s->h;
    if (B > 1 && (lam_stride < 2 * (int64_t)h.nn || v_stride < h.n ||
                  (type_stride != 0 && type_stride < h.n) ||
                  (branch_stride != 0 && branch_stride < h.m) ||
                  (bus && d_gP && d_gQ && g_stride < h.n)))
        return fail(PF_E_WORKSPACE, "pf_adjoint_params: a stride is too small");
    if (B == 0) return PF_OK;
    if (bus && d_gP && d_gQ) {
        dim3 grid((s->h.n + 255) / 256, B);
        hipLaunchKernelGGL(k_adj_bus, grid, dim3(256), 0, as_stream(stream), s->h.dev, d_lam,
                           lam_stride, d_type, type_stride, d_gP, d_gQ, g_stride);
        int rc = launch_check("pf_adjoint_params");
        if (rc) return rc;
    }
    if (d_gx && s->h.m > 0) {
        if (!d_r || !d_x) return fail(PF_E_INVALID, "pf_adjoint_params: need r and x");
        const dim3 grid(gx_mode == 1 ? (s->h.m + 63) / 64 : (s->h.m + 255) / 256,
                        gx_mode == 1 ? 1 : B);
        const dim3 block(gx_mode == 1 ? 1024 : 256);
        hipLaunchKernelGGL(k_adj_branch, grid, block, 0, as_stream(stream), s->h.dev,
                           s->d_from, s->d_to, B, d_lam, lam_stride, d_type, type_stride, d_Vm,
                           d_Va, v_stride, d_r, d_x, branch_stride, d_status, d_gx, gx_mode);
        return launch_check("pf_adjoint_params");
    }
    return PF_OK;
}
}  // namespace abi
}  // namespace pf

extern "C" {

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
    std::vector<int64_t>& work = p->work;
    work.assign(G, 0);
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
    plan_blocks(p);
    *out = p;
    return PF_OK;
}

int pf_multi_set_spread(pf_multi p, int workgroups)
{
    if (!p) return fail(PF_E_INVALID, "pf_multi_set_spread: NULL plan");
    if (workgroups < 0 || workgroups > 65535)
        return fail(PF_E_INVALID, "pf_multi_set_spread: workgroups must be 0..65535");
    p->spread = workgroups;
    plan_blocks(p);
    p->uploaded = false;  // the block table on the device is stale: upload again
    return PF_OK;
}

int pf_multi_info(const pf_multi p, size_t* dev_bytes, int64_t* bus_off, int64_t* branch_off,
                  int64_t* y_off, int64_t* ws_off)
{
    if (!p) return fail(PF_E_INVALID, "pf_multi_info: NULL plan");
    size_t G = p->syms.size();
    if (dev_bytes)
        *dev_bytes = ((G * sizeof(CaseDesc) + 255) & ~(size_t)255) +
                     ((std::max<size_t>(G, 1) * 4 + 255) & ~(size_t)255) +
                     ((p->blocks.size() * 4 + 255) & ~(size_t)255);
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
    p->uploaded = false;
    p->gens.assign(G, 0);
    for (size_t g = 0; g < G; ++g) {
        if (!p->syms[g]->h.uploaded)
            return fail(PF_E_INVALID, "pf_multi_upload: a symbolic is not uploaded");
        cd[g].sym = p->syms[g]->h.dev;
        p->gens[g] = p->syms[g]->h.upload_gen;
        cd[g].bus_off = p->bus_off[g];
        cd[g].br_off = p->br_off[g];
        cd[g].y_off = p->y_off[g];
        cd[g].ws_off = p->ws_off[g];
        cd[g].sync_off = p->syms[g]->h.sync_off();
        cd[g].spread = p->counts[g];
        cd[g].back_lo = spread_back_lo(p->syms[g]->h, multi_threads(p));
    }
    size_t ooff = (G * sizeof(CaseDesc) + 255) & ~(size_t)255;
    if (G) std::memcpy(stage.data() + ooff, p->order.data(), G * sizeof(int32_t));
    const size_t boff = ooff + ((std::max<size_t>(G, 1) * 4 + 255) & ~(size_t)255);
    if (!p->blocks.empty())
        std::memcpy(stage.data() + boff, p->blocks.data(), p->blocks.size() * sizeof(int32_t));
    int rc = hip_check(hipMemcpyAsync(d_buf, stage.data(), need, hipMemcpyHostToDevice,
                                      as_stream(stream)),
                       "pf_multi_upload: hipMemcpyAsync");
    if (rc) return rc;
    rc = hip_check(hipStreamSynchronize(as_stream(stream)), "pf_multi_upload: sync");
    if (rc) return rc;
    p->d_desc = reinterpret_cast<const CaseDesc*>(d_buf);
    p->d_order = reinterpret_cast<const int32_t*>(static_cast<char*>(d_buf) + ooff);
    p->d_blocks = reinterpret_cast<const int4*>(static_cast<char*>(d_buf) + boff);
    p->uploaded = true;
    return PF_OK;
}

// A plan whose members were all uploaded as they are now (else the descriptors
// it copied to the device are stale).
static bool plan_current(const pf_multi p, const char* fn)
{
    if (!p || !p->uploaded) {
        fail(PF_E_INVALID, std::string(fn) + ": plan not uploaded");
        return false;
    }
    for (size_t g = 0; g < p->syms.size(); ++g) {
        const HostSym& h = p->syms[g]->h;
        if (!h.uploaded || h.upload_gen != p->gens[g]) {
            fail(PF_E_INVALID, std::string(fn) + ": symbolic " + std::to_string(g) +
                                   " changed since pf_multi_upload; upload the plan again");
            return false;
        }
    }
    return true;
}

int pf_build_ybus_multi(const pf_multi p, const double* d_r, const double* d_x,
                        const double* d_b, const double* d_ysh, double* d_yval, void* stream)
{
    if (!plan_current(p, "pf_build_ybus_multi")) return PF_E_INVALID;
    if (!d_r || !d_x || !d_b || !d_yval) return fail(PF_E_INVALID, "pf_build_ybus_multi: NULL");
    if (d_ysh && (reinterpret_cast<uintptr_t>(d_ysh) & 15))
        return fail(PF_E_INVALID, "pf_build_ybus_multi: d_ysh must be 16-byte aligned");
    if (p->syms.empty()) return PF_OK;
    // enough workgroups per case for the largest grid's rows, at most 256
    int nmax = 0;
    for (auto* sy : p->syms) nmax = std::max(nmax, sy->h.n);
    const int per = (int)std::max<int64_t>(
        1, std::min<int64_t>(256, ((int64_t)nmax * kYbusLanes + 255) / 256));
    hipLaunchKernelGGL(k_ybus_multi, dim3((unsigned)p->syms.size(), per), dim3(256), 0,
                       as_stream(stream), p->d_desc, d_r, d_x, d_b, d_ysh, d_yval);
    return launch_check("pf_build_ybus_multi");
}

int pf_newton_multi(const pf_multi p, const double* d_yval, const int8_t* d_type,
                    const double* d_Psp, const double* d_Qsp, double* d_Vm, double* d_Va,
                    double tol, int max_iter, int flags, double* d_ws, int32_t* d_iters,
                    double* d_norm, int32_t* d_status, int32_t* d_pivot, void* stream)
{
    if (!plan_current(p, "pf_newton_multi")) return PF_E_INVALID;
    if (max_iter < 0 || !(tol >= 0.0) || !d_yval || !d_type || !d_Psp || !d_Qsp || !d_Vm ||
        !d_Va || !d_ws)
        return fail(PF_E_INVALID, "pf_newton_multi: bad arguments");
    if (reinterpret_cast<uintptr_t>(d_ws) & 15)
        return fail(PF_E_WORKSPACE, "pf_newton_multi: workspace must be 16-byte aligned");
    if (p->syms.empty()) return PF_OK;
    NewtonArgs a{d_yval, 0, d_type, 0, d_Psp, d_Qsp, 0, d_Vm, d_Va, 0, d_ws, 0, tol, max_iter,
                 flags, 1, (int)p->syms.size(), d_iters, d_norm, d_status, d_pivot};
    DevSym none{};
    int lds = 0;
    uint64_t wait = 0;
    for (auto* sy : p->syms) {
        lds = std::max(lds, newton_lds(sy->h));
        wait = std::max<uint64_t>(wait, sy->h.spread_wait);
    }
    const int threads = multi_threads(p);
    allow_big_lds();
    const int G = (int)p->syms.size();
    const int nb = (int)p->blocks.size() / 4;
    hipStream_t st = as_stream(stream);
    if (nb > G) {
        // more workgroups than cases: one cooperative launch, when the device
        // keeps them all resident and the stream is not being captured
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        int dev = 0, cus = 0, per = 0;
        const bool queried =
            hipStreamIsCapturing(st, &cs) == hipSuccess && hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) ==
                hipSuccess &&
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_newton_multi_spread, threads,
                                                         lds) == hipSuccess;
        if (!queried) (void)hipGetLastError();
        if (queried && cs == hipStreamCaptureStatusNone && nb <= per * cus) {
            hipLaunchKernelGGL(k_spread_init_multi, dim3(G), dim3(128), 0, st, p->d_desc, d_ws);
            if (const int e = launch_check("pf_newton_multi")) return e;
            const CaseDesc* descs = p->d_desc;
            const int4* blocks = p->d_blocks;
            unsigned long long w = wait;
            void* args[] = {&descs, &blocks, &a, &w};
            return hip_check(
                hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_newton_multi_spread),
                                           dim3(nb), dim3(threads), args, (unsigned)lds, st),
                "pf_newton_multi");
        }
    }
    hipLaunchKernelGGL(k_newton<true>, dim3(G), dim3(threads), lds, st, none, p->d_desc,
                       p->d_order, a);
    return launch_check("pf_newton_multi");
}

void pf_multi_destroy(pf_multi p) { delete p; }

}  // extern "C"
