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
//   k_fd_*, k_fdpf  fast decoupled matrices, LDL^T, iteration       [III, Table III]
//   k_branch_flows  post-convergence branch flows                   [II-A]
//   k_se_*        WLS state estimation: state, measurements, gain   [IV]
//
// Work decomposition inside a workgroup: hierarchical levels run one after
// the other with a workgroup barrier between them; inside a level, each
// node gets a group of g lanes (g from the symbolic's per-level mapping);
// the lanes of a group split the node's destinations and its descendant
// list, and combine partial sums with a butterfly over the group.  The top
// levels whose values fit (the "tail") run in LDS, the top clique of the
// elimination tree as a dense block.  Outside the tail the Newton and fast
// decoupled kernels reuse the same LDS for a copy of every bus's (e, f)
// (mismatch, Jacobian) and for the sweeps' solution vector.
//
// Memory layout across cases: a batch is cut into groups of C cases whose
// per-case arrays are interleaved in chunks (64 bytes for filled values: one
// slot record or two diagonal blocks; 32 bytes for bus records and the
// rhs), so one 128-byte line holds the same record of two or four cases.
// The C workgroups of a group are launched 8 blocks apart, which places them
// on the same XCD at the same time: they walk the same pattern in near
// lockstep and share every line they fetch through that XCD's L2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <numeric>
#include <string>
#include <type_traits>
#include <vector>

#include "pf.h"
#include "pf_internal.h"
#include "pf_kernels.h"

using namespace pf;

// ===========================================================================
// device helpers
// ===========================================================================
extern __shared__ double pf_smem[];  // dynamic LDS: tail, (e, f) copy, vectors, PV mask

namespace {

constexpr int kMaxThreads = 1024;
// The level-scheduled kernels are bounded at 512 threads per workgroup, which
// leaves them 256 VGPRs per lane: their per-node working set (two 2x2
// destination pairs, prefetched records, reduction partials) then fits in
// registers without spilling.
constexpr int kLevelThreads = 512;
constexpr int kXcds = 8;
constexpr int kWave = 64;  // CDNA wavefront
constexpr size_t kSolveLdsMax = 159 * 1024;  // of the 160 KB of LDS per workgroup on gfx950

// Orders the LDS accesses of one wavefront's lanes (they run in lockstep,
// and a wavefront's LDS operations are performed in issue order).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One case's doubles inside an interleaved group of C cases: element d
// lives at base + (d / K) * K C + K (case % C) + d % K, i.e. chunks of K
// doubles of the C cases alternate.  The filled values use K = 8 (a slot
// record W, U is one 64-byte chunk, in a single cache line); the Newton
// bus records and rhs use K = 4 (the 32-byte voltage part of a bus record,
// which is what neighbours gather, shares its line with three other
// cases' only).  C = 1 is the plain contiguous layout.
struct View {
    double* base;
    int lane;  // K * (case % C)
    int sh;    // log2(K C)
    int cs;    // log2(K)
    __device__ __forceinline__ double* at(int64_t d) const
    {
        return base + ((d >> cs) << sh) + lane + (d & ((1 << cs) - 1));
    }
    __device__ __forceinline__ Blk blk(int64_t d) const { return bload(at(d)); }
    __device__ __forceinline__ void put(int64_t d, const Blk& v) const { bstore(at(d), v); }
    __device__ __forceinline__ double2 v2(int64_t d) const
    {
        return *reinterpret_cast<const double2*>(at(d));
    }
    __device__ __forceinline__ void put2(int64_t d, double2 v) const
    {
        *reinterpret_cast<double2*>(at(d)) = v;
    }
};

__device__ __forceinline__ int ilog2(int c) { return 31 - __clz(c); }

// Case of block b when groups of C cases are placed 8 blocks apart (same
// XCD under the round-robin workgroup dispatch); -1 for padding blocks.
__device__ __forceinline__ int case_of_block(int b, int C, int B)
{
    int c = b;
    if (C > 1) {
        const int span = kXcds * C;
        const int hi = b / span, rem = b - hi * span;
        c = (hi * kXcds + (rem & (kXcds - 1))) * C + rem / kXcds;
    }
    return c < B ? c : -1;
}

// Filled values of case c (64-byte chunks).
__device__ __forceinline__ View case_view(double* buf, int64_t stride, int C, int c)
{
    View v;
    v.base = buf + (int64_t)(c / C) * C * stride;
    v.lane = 8 * (c % C);
    v.sh = 3 + ilog2(C);
    v.cs = 3;
    return v;
}

// The Newton workspace's part after the filled values (bus records, rhs) of
// case c, offsets relative to its start (32-byte chunks).
__device__ __forceinline__ View case_bus_view(double* buf, int64_t stride, int C, int c,
                                              int64_t vals)
{
    View v;
    v.base = buf + (int64_t)(c / C) * C * stride + vals * C;
    v.lane = 4 * (c % C);
    v.sh = 2 + ilog2(C);
    v.cs = 2;
    return v;
}

// Offsets of the Newton workspace of one case (doubles):
//   D [nn][4] (padded) | LU [nnz_l][8] | bus records [n][8] | rhs [nn][2]
// D and LU through the values view; BUS and RHS relative to the bus view.
// bus record: e, f, |V|, theta | P, Q, -, -  (e + jf = V, P + jQ = S).
struct Off {
    int64_t D, LU, BUS, RHS;
};
__device__ __forceinline__ Off ws_off(const DevSym& S)
{
    Off o;
    o.D = 0;
    o.LU = S.lu_off;
    o.BUS = 0;
    o.RHS = 8 * (int64_t)S.n;
    return o;
}

// Voltage accessors: stored rectangular voltages, or computed from polar.
struct EFView {
    View v;
    int64_t bus_off;
    __device__ __forceinline__ void get(int k, double& ek, double& fk) const
    {
        const double2 t = v.v2(bus_off + 8 * (int64_t)k);
        ek = t.x;
        fk = t.y;
    }
};
// (e, f) of every bus copied into LDS (the Newton mismatch pass).
struct EFLds {
    double2* s;
    __device__ __forceinline__ void get(int k, double& ek, double& fk) const
    {
        const double2 t = s[k];
        ek = t.x;
        fk = t.y;
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

// P_i + jQ_i = V_i conj(sum_k Y_ik V_k)  (nodal: one row of Y, entries
// [q0, q1), summed in order).  The first four entries' indices, admittances
// and voltages are requested together (in-bounds loads of entry q0 stand in
// for absent ones), the rest two at a time.
template <class EF>
__device__ __forceinline__ void injection_row(const DevSym& S, const double* __restrict__ yv,
                                              const EF& ef, int i, int q0, int q1, double& P,
                                              double& Q)
{
    const double2* y2 = reinterpret_cast<const double2*>(yv);
    double ei, fi;
    ef.get(i, ei, fi);
    int kq[4];
    double2 yq[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int q = q0 + k < q1 ? q0 + k : q0;
        kq[k] = S.ycol[q];
        yq[k] = y2[q];
    }
    double ek[4], fk[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) ef.get(kq[k], ek[k], fk[k]);
    double ir = 0.0, ii = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (q0 + k < q1) {
            ir = fma(yq[k].x, ek[k], fma(-yq[k].y, fk[k], ir));
            ii = fma(yq[k].x, fk[k], fma(yq[k].y, ek[k], ii));
        }
    }
    int q = q0 + 4;
    for (; q + 1 < q1; q += 2) {
        const int k0 = S.ycol[q], k1 = S.ycol[q + 1];
        const double2 y0 = y2[q], y1 = y2[q + 1];
        double e0, f0, e1, f1;
        ef.get(k0, e0, f0);
        ef.get(k1, e1, f1);
        ir = fma(y0.x, e0, fma(-y0.y, f0, ir));
        ii = fma(y0.x, f0, fma(y0.y, e0, ii));
        ir = fma(y1.x, e1, fma(-y1.y, f1, ir));
        ii = fma(y1.x, f1, fma(y1.y, e1, ii));
    }
    if (q < q1) {
        const int k0 = S.ycol[q];
        const double2 y0 = y2[q];
        double e0, f0;
        ef.get(k0, e0, f0);
        ir = fma(y0.x, e0, fma(-y0.y, f0, ir));
        ii = fma(y0.x, f0, fma(y0.y, e0, ii));
    }
    P = ei * ir + fi * ii;
    Q = fi * ir - ei * ii;
}

template <class EF>
__device__ __forceinline__ void injection(const DevSym& S, const double* __restrict__ yv,
                                          const EF& ef, int i, double& P, double& Q)
{
    injection_row(S, yv, ef, i, S.yptr[i], S.yptr[i + 1], P, Q);
}

// PV flags of one case's buses, one bit per bus, in LDS after the tail.
struct PvMask {
    const uint32_t* m;
    __device__ __forceinline__ bool operator()(int k) const { return (m[k >> 5] >> (k & 31)) & 1u; }
};

__device__ __forceinline__ uint32_t* pv_words(const DevSym& S)
{
    const int off = S.tail_lds > S.ef_lds ? S.tail_lds : S.ef_lds;
    return reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(pf_smem) + off);
}

// Fills the mask m from the case's bus types (a ballot per wavefront); the
// caller synchronises before use.
__device__ __forceinline__ void pv_fill_at(uint32_t* m, const DevSym& S, const int8_t* type)
{
    for (int base = 0; base < S.n; base += blockDim.x) {
        const int i = base + threadIdx.x;
        const unsigned long long bits = __ballot(i < S.n && type[i] == T_PV);
        if ((threadIdx.x & 63) == 0 && i < S.n) {
            m[i >> 5] = (uint32_t)bits;
            m[(i >> 5) + 1] = (uint32_t)(bits >> 32);
        }
    }
}

__device__ __forceinline__ void pv_fill(const DevSym& S, const int8_t* type)
{
    pv_fill_at(pv_words(S), S, type);
}

// First four admittance entries of one row: indices and values, then the
// voltages they multiply (two dependent batches of loads, no stores).
struct RowHead {
    double2 y[4];
    double e[4], f[4];
};

template <class EF>
__device__ __forceinline__ void row_head_idx(const DevSym& S, const double* __restrict__ yv,
                                             int q0, int q1, int (&k)[4], RowHead& h)
{
    const double2* y2 = reinterpret_cast<const double2*>(yv);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int q = q0 + t < q1 ? q0 + t : q0;
        k[t] = S.ycol[q];
        h.y[t] = y2[q];
    }
}

template <class EF>
__device__ __forceinline__ void row_head_v(const EF& ef, const int (&k)[4], RowHead& h)
{
#pragma unroll
    for (int t = 0; t < 4; ++t) ef.get(k[t], h.e[t], h.f[t]);
}

// Sum of the row (head from registers, the rest loaded two at a time), in
// entry order, and the injection at bus voltage (ei, fi).
template <class EF>
__device__ __forceinline__ void row_finish(const DevSym& S, const double* __restrict__ yv,
                                           const EF& ef, int q0, int q1, const RowHead& h,
                                           double ei, double fi, double& P, double& Q)
{
    const double2* y2 = reinterpret_cast<const double2*>(yv);
    double ir = 0.0, ii = 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        if (q0 + t < q1) {
            ir = fma(h.y[t].x, h.e[t], fma(-h.y[t].y, h.f[t], ir));
            ii = fma(h.y[t].x, h.f[t], fma(h.y[t].y, h.e[t], ii));
        }
    }
    int q = q0 + 4;
    for (; q + 1 < q1; q += 2) {
        const int k0 = S.ycol[q], k1 = S.ycol[q + 1];
        const double2 y0 = y2[q], y1 = y2[q + 1];
        double e0, f0, e1, f1;
        ef.get(k0, e0, f0);
        ef.get(k1, e1, f1);
        ir = fma(y0.x, e0, fma(-y0.y, f0, ir));
        ii = fma(y0.x, f0, fma(y0.y, e0, ii));
        ir = fma(y1.x, e1, fma(-y1.y, f1, ir));
        ii = fma(y1.x, f1, fma(y1.y, e1, ii));
    }
    if (q < q1) {
        const int k0 = S.ycol[q];
        const double2 y0 = y2[q];
        double e0, f0;
        ef.get(k0, e0, f0);
        ir = fma(y0.x, e0, fma(-y0.y, f0, ir));
        ii = fma(y0.x, f0, fma(y0.y, e0, ii));
    }
    P = ei * ir + fi * ii;
    Q = fi * ir - ei * ii;
}

// Jacobian source: the Newton state of one case (bus records in the view).
// diag_in / off_in only issue loads, diag_of / off_of only compute, so that a
// caller can have all of a node's loads in flight before it waits for any.
// Invalid indices are never dereferenced: a fill slot (no admittance entry)
// reads entry 0 and is then zeroed.
struct SrcState {
    const double* yv;
    PvMask type;
    View w;
    int64_t bus_off;
    // (e, f) of every bus in LDS, or null: diag_in / off_in then read (e, f)
    // there and |V| is taken as sqrt(e^2 + f^2)
    const double2* efs;
    struct DiagIn {
        double2 y;
        Blk r;  // e, f, |V|, theta of the node's bus
        double2 s;
        bool pv;
    };
    struct OffIn {
        Blk rk;
        double2 yl, yu;
        bool pk, fill;
    };
    __device__ __forceinline__ DiagIn diag_in(int, int bus, int yd) const
    {
        const double2* y2 = reinterpret_cast<const double2*>(yv);
        const int64_t rec = bus_off + 8 * (int64_t)bus;
        Blk r;
        if (efs) {
            const double2 t = efs[bus];
            r = {t.x, t.y, 0.0, 0.0};
        } else {
            r = w.blk(rec);
        }
        return {y2[yd], r, w.v2(rec + 4), type(bus)};
    }
    __device__ __forceinline__ double vm_of(const Blk& r) const
    {
        return efs ? sqrt(fma(r.a, r.a, r.b * r.b)) : r.c;
    }
    __device__ __forceinline__ Blk diag_of(const DiagIn& d) const
    {
        return jac_diag(d.y.x, d.y.y, d.s.x, d.s.y, vm_of(d.r), d.pv);
    }
    __device__ __forceinline__ OffIn off_in(int, int bk, int ylo, int yup) const
    {
        const double2* y2 = reinterpret_cast<const double2*>(yv);
        const bool fill = ylo < 0;
        Blk rk;
        if (efs) {
            const double2 t = efs[bk];
            rk = {t.x, t.y, 0.0, 0.0};
        } else {
            rk = w.blk(bus_off + 8 * (int64_t)bk);
        }
        return {rk, y2[fill ? 0 : ylo], y2[fill ? 0 : yup], type(bk), fill};
    }
    __device__ __forceinline__ void off_of(const DiagIn& dj, const OffIn& o, Blk& lo,
                                           Blk& up) const
    {
        if (o.fill) {
            lo = bzero();
            up = bzero();
            return;
        }
        const double vk = vm_of(o.rk);
        lo = jac_off(o.yl.x, o.yl.y, o.rk.a, o.rk.b, dj.r.a, dj.r.b, vm_of(dj.r), o.pk, dj.pv);
        up = jac_off(o.yu.x, o.yu.y, dj.r.a, dj.r.b, o.rk.a, o.rk.b, vk, dj.pv, o.pk);
    }
    __device__ __forceinline__ Blk diag(int, int bus, int yd) const
    {
        const double2 y = reinterpret_cast<const double2*>(yv)[yd];
        const double vm = *w.at(bus_off + 8 * (int64_t)bus + 2);
        const double2 s = w.v2(bus_off + 8 * (int64_t)bus + 4);
        return jac_diag(y.x, y.y, s.x, s.y, vm, type(bus));
    }
    // block (k, j) below the diagonal and (j, k) above it; zero at fill
    __device__ __forceinline__ void off(int, int bj, int bk, int ylo, int yup, Blk& lo,
                                        Blk& up) const
    {
        if (ylo < 0) {
            lo = bzero();
            up = bzero();
            return;
        }
        const Blk rj = w.blk(bus_off + 8 * (int64_t)bj);  // e, f, |V|, theta
        const Blk rk = w.blk(bus_off + 8 * (int64_t)bk);
        const bool pj = type(bj), pk = type(bk);
        const double2 yl = reinterpret_cast<const double2*>(yv)[ylo];
        const double2 yu = reinterpret_cast<const double2*>(yv)[yup];
        lo = jac_off(yl.x, yl.y, rk.a, rk.b, rj.a, rj.b, rj.c, pk, pj);
        up = jac_off(yu.x, yu.y, rj.a, rj.b, rk.a, rk.b, rk.c, pj, pk);
    }
};

// Jacobian source: an assembled matrix in the filled layout.
// LOWER_ONLY (a symmetric matrix, factorised with the upper factor taken
// from the lower one): off_in reads the lower block alone.
template <bool LOWER_ONLY>
struct SrcLoadT {
    View w;
    int64_t lu_off;
    struct DiagIn {
        Blk a;
    };
    struct OffIn {
        Blk lo, up;
    };
    __device__ __forceinline__ DiagIn diag_in(int j, int, int) const
    {
        return {w.blk(4 * (int64_t)j)};
    }
    __device__ __forceinline__ Blk diag_of(const DiagIn& d) const { return d.a; }
    __device__ __forceinline__ OffIn off_in(int s, int, int, int) const
    {
        return {w.blk(lu_off + 8 * (int64_t)s),
                LOWER_ONLY ? bzero() : w.blk(lu_off + 8 * (int64_t)s + 4)};
    }
    __device__ __forceinline__ void off_of(const DiagIn&, const OffIn& o, Blk& lo,
                                           Blk& up) const
    {
        lo = o.lo;
        up = o.up;
    }
    __device__ __forceinline__ Blk diag(int j, int, int) const { return w.blk(4 * (int64_t)j); }
    __device__ __forceinline__ void off(int s, int, int, int, int, Blk& lo, Blk& up) const
    {
        lo = w.blk(lu_off + 8 * (int64_t)s);
        up = w.blk(lu_off + 8 * (int64_t)s + 4);
    }
};
using SrcLoad = SrcLoadT<false>;

// Runs fn(x, lane, g) for the nodes of levels [l0, l1), x indexing the
// level-ordered node records, up or down, with a barrier after every level.
template <class F>
__device__ __forceinline__ void for_levels(const DevSym& S, int l0, int l1, bool up, F&& fn)
{
    for (int li = l0; li < l1; ++li) {
        const int l = up ? li : l1 - 1 - (li - l0);
        const int g = S.level_g[l];
        const int beg = S.level_ptr[l];
        const int cnt = S.level_ptr[l + 1] - beg;
        const int gpb = blockDim.x / g;
        const int grp = threadIdx.x / g;
        const int lane = threadIdx.x & (g - 1);
        for (int base = 0; base < cnt; base += gpb) {
            const int idx = base + grp;
            if (idx < cnt) fn(beg + idx, lane, g);
        }
        __syncthreads();
    }
}

// Level-ordered node record, the part the sweeps use ({j, bus, r0, r1},
// {s0, s1, ydiag, 0}); the admittance-row range is read by the mismatch only.
struct NodeRec {
    int4 a, b;
};

__device__ __forceinline__ NodeRec load_rec(const DevSym& S, int x)
{
    return {S.node_info[3 * x], S.node_info[3 * x + 1]};
}

// As for_levels, passing fn(x, rec, lane, g) the node's record; the record
// of the group's next node in the level is fetched before fn runs so that
// its latency overlaps the current node's work.
template <class F>
__device__ __forceinline__ void for_nodes(const DevSym& S, int l0, int l1, bool up, F&& fn)
{
    for (int li = l0; li < l1; ++li) {
        const int l = up ? li : l1 - 1 - (li - l0);
        const int g = S.level_g[l];
        const int beg = S.level_ptr[l];
        const int cnt = S.level_ptr[l + 1] - beg;
        const int gpb = blockDim.x / g;
        const int grp = threadIdx.x / g;
        const int lane = threadIdx.x & (g - 1);
        int idx = grp;
        NodeRec cur = idx < cnt ? load_rec(S, beg + idx) : NodeRec{};
        while (idx < cnt) {
            const int nxt = idx + gpb;
            const NodeRec pre = nxt < cnt ? load_rec(S, beg + nxt) : NodeRec{};
            fn(beg + idx, cur, lane, g);
            cur = pre;
            idx = nxt;
        }
        __syncthreads();
    }
}

// Runs fn(jl, lane, g) over tail levels [t0, t1) (tail-local numbering).
template <class F>
__device__ __forceinline__ void for_tail_range(const DevSym& S, int t0, int t1, bool up, F&& fn)
{
    for (int ti = t0; ti < t1; ++ti) {
        const int tl = up ? ti : t1 - 1 - (ti - t0);
        const int g = S.level_g[S.tail_level + tl];
        const int beg = S.t_lptr[tl];
        const int cnt = S.t_lptr[tl + 1] - beg;
        const int gpb = blockDim.x / g;
        const int grp = threadIdx.x / g;
        const int lane = threadIdx.x & (g - 1);
        for (int base = 0; base < cnt; base += gpb) {
            const int idx = base + grp;
            if (idx < cnt) fn(beg + idx, lane, g);
        }
        __syncthreads();
    }
}

// As for_tail_range, passing fn(jl, the three parts of t_node[jl], lane, g);
// each thread's first record of the next level is requested before the
// barrier that ends the current one, so it is in registers when that level
// starts.
template <class F>
__device__ __forceinline__ void for_tail_pf(const DevSym& S, int t0, int t1, bool up, F&& fn)
{
    if (t0 >= t1) return;
    int g = 1, beg = 0, cnt = 0;
    int4 ra = make_int4(0, 0, 0, 0), rb = ra, rc = ra;
    auto fetch = [&](int tl) {
        g = S.level_g[S.tail_level + tl];
        beg = S.t_lptr[tl];
        cnt = S.t_lptr[tl + 1] - beg;
        const int idx = threadIdx.x / g;
        const int jl = beg + (idx < cnt ? idx : 0);
        ra = S.t_node[3 * jl];
        rb = S.t_node[3 * jl + 1];
        rc = S.t_node[3 * jl + 2];
    };
    fetch(up ? t0 : t1 - 1);
    for (int ti = t0; ti < t1; ++ti) {
        const int gg = g, b0 = beg, c0 = cnt;
        const int4 a0 = ra, a1 = rb, a2 = rc;
        if (ti + 1 < t1) fetch(up ? ti + 1 : t1 - 2 - (ti - t0));
        const int gpb = blockDim.x / gg, grp = threadIdx.x / gg, lane = threadIdx.x & (gg - 1);
        for (int base = 0; base < c0; base += gpb) {
            const int idx = base + grp;
            if (idx >= c0) continue;
            const int jl = b0 + idx;
            if (base == 0) fn(jl, a0, a1, a2, lane, gg);
            else fn(jl, S.t_node[3 * jl], S.t_node[3 * jl + 1], S.t_node[3 * jl + 2], lane, gg);
        }
        __syncthreads();
    }
}

// Block updates of one destination slot from pairs (a, b) = (slot(i;k), slot(i;j)):
//   W_kj -= W_ki U_ij,  V_jk -= W_ji U_ik.
// Two pairs per step; the next step's indices are fetched before this
// step's blocks so that index and value loads overlap.  Absent pairs read
// entry 0 (always in bounds) and contribute nothing.
__device__ __forceinline__ int2 upd_at(const int2* __restrict__ upd, int u, int u1)
{
    return upd[u < u1 ? u : 0];
}

__device__ __forceinline__ void apply_updates(const int2* __restrict__ upd, int u0, int u1,
                                              const View& w, int64_t lu, Blk& Wk, Blk& Vk)
{
    if (u0 >= u1) return;
    int2 p = upd[u0];
    int2 q = upd_at(upd, u0 + 1, u1);
    for (int u = u0; u < u1; u += 2) {
        const bool has_q = u + 1 < u1;
        const int2 pn = upd_at(upd, u + 2, u1);
        const int2 qn = upd_at(upd, u + 3, u1);
        const Blk Wa = w.blk(lu + 8 * (int64_t)p.x), Ua = w.blk(lu + 8 * (int64_t)p.x + 4);
        const Blk Wb = w.blk(lu + 8 * (int64_t)p.y), Ub = w.blk(lu + 8 * (int64_t)p.y + 4);
        const Blk Wc = w.blk(lu + 8 * (int64_t)q.x), Uc = w.blk(lu + 8 * (int64_t)q.x + 4);
        const Blk Wd = w.blk(lu + 8 * (int64_t)q.y), Ud = w.blk(lu + 8 * (int64_t)q.y + 4);
        bmsub(Wk, Wa, Ub);
        bmsub(Vk, Wb, Ua);
        if (has_q) {
            bmsub(Wk, Wc, Ud);
            bmsub(Vk, Wd, Uc);
        }
        p = pn;
        q = qn;
    }
}

// The updates of two destinations at once, one pair of each per step, with
// the first pairs (p, q) already loaded: both chains of loads are in flight
// together.  The order of the updates of each destination is the list order.
// SYM (symmetric matrix): only W is updated (V_jk = W_kj^T throughout), so
// each pair reads two blocks instead of four.
template <bool SYM = false>
__device__ __forceinline__ void apply_updates2(const int2* __restrict__ upd, int u0, int u1,
                                               int v0, int v1, int2 p, int2 q, const View& w,
                                               int64_t lu, Blk& Wk, Blk& Vk, Blk& Wk2, Blk& Vk2)
{
    for (int a = u0, b = v0; a < u1 || b < v1; ++a, ++b) {
        const bool hp = a < u1, hq = b < v1;
        const int2 pn = upd_at(upd, a + 1, u1);
        const int2 qn = upd_at(upd, b + 1, v1);
        if (SYM) {
            const Blk Wa = w.blk(lu + 8 * (int64_t)p.x), Ub = w.blk(lu + 8 * (int64_t)p.y + 4);
            const Blk Wc = w.blk(lu + 8 * (int64_t)q.x), Ud = w.blk(lu + 8 * (int64_t)q.y + 4);
            if (hp) bmsub(Wk, Wa, Ub);
            if (hq) bmsub(Wk2, Wc, Ud);
        } else {
            const Blk Wa = w.blk(lu + 8 * (int64_t)p.x), Ua = w.blk(lu + 8 * (int64_t)p.x + 4);
            const Blk Wb = w.blk(lu + 8 * (int64_t)p.y), Ub = w.blk(lu + 8 * (int64_t)p.y + 4);
            const Blk Wc = w.blk(lu + 8 * (int64_t)q.x), Uc = w.blk(lu + 8 * (int64_t)q.x + 4);
            const Blk Wd = w.blk(lu + 8 * (int64_t)q.y), Ud = w.blk(lu + 8 * (int64_t)q.y + 4);
            if (hp) {
                bmsub(Wk, Wa, Ub);
                bmsub(Vk, Wb, Ua);
            }
            if (hq) {
                bmsub(Wk2, Wc, Ud);
                bmsub(Vk2, Wd, Uc);
            }
        }
        p = pn;
        q = qn;
    }
}

// Same with the blocks in LDS (tail-local slot numbering).
__device__ __forceinline__ void apply_updates_lds(const int2* __restrict__ upd, int u0, int u1,
                                                  const double* sLU, Blk& Wk, Blk& Vk)
{
    if (u0 >= u1) return;
    int2 p = upd[u0];
    int2 q = (u0 + 1 < u1) ? upd[u0 + 1] : make_int2(0, 0);
    for (int u = u0; u < u1; u += 2) {
        const bool has_q = u + 1 < u1;
        const int2 pn = (u + 2 < u1) ? upd[u + 2] : make_int2(0, 0);
        const int2 qn = (u + 3 < u1) ? upd[u + 3] : make_int2(0, 0);
        bmsub(Wk, bload(sLU + 8 * p.x), bload(sLU + 8 * p.y + 4));
        bmsub(Vk, bload(sLU + 8 * p.y), bload(sLU + 8 * p.x + 4));
        if (has_q) {
            bmsub(Wk, bload(sLU + 8 * q.x), bload(sLU + 8 * q.y + 4));
            bmsub(Vk, bload(sLU + 8 * q.y), bload(sLU + 8 * q.x + 4));
        }
        p = pn;
        q = qn;
    }
}

// Word k of a 16-byte load of a packed list.
__device__ __forceinline__ uint32_t pk_word(const uint4& q, int k)
{
    return k == 0 ? q.x : k == 1 ? q.y : k == 2 ? q.z : q.w;
}

// Updates of two tail destinations from their packed local pair lists
// (n1, n2 pairs starting at loads l1, l2; words (slot(i;k), slot(i;j))):
// four pairs of each per step, the next step's loads in flight.  The order
// of the updates of each destination is the list order.
__device__ __forceinline__ void apply_packed2_lds(const uint4* __restrict__ pk, int l1, int n1,
                                                  int l2, int n2, const double* sLU, Blk& Wk,
                                                  Blk& Vk, Blk& Wk2, Blk& Vk2)
{
    uint4 q1 = pk[n1 > 0 ? l1 : 0], q2 = pk[n2 > 0 ? l2 : 0];
    for (int k = 0; k < n1 || k < n2; k += 4) {
        const int i = (k >> 2) + 1;
        const uint4 q1n = pk[k + 4 < n1 ? l1 + i : 0];
        const uint4 q2n = pk[k + 4 < n2 ? l2 + i : 0];
        // one pair of each destination in flight at a time (register budget)
#pragma unroll 1
        for (int c = 0; c < 4; ++c) {
            if (k + c < n1) {
                const uint32_t v = pk_word(q1, c);
                const int a = v & 0xffff, b = v >> 16;
                bmsub(Wk, bload(sLU + 8 * a), bload(sLU + 8 * b + 4));
                bmsub(Vk, bload(sLU + 8 * b), bload(sLU + 8 * a + 4));
            }
            if (k + c < n2) {
                const uint32_t v = pk_word(q2, c);
                const int a = v & 0xffff, b = v >> 16;
                bmsub(Wk2, bload(sLU + 8 * a), bload(sLU + 8 * b + 4));
                bmsub(Vk2, bload(sLU + 8 * b), bload(sLU + 8 * a + 4));
            }
        }
        q1 = q1n;
        q2 = q2n;
    }
}

__device__ __forceinline__ void gsum_blk(Blk& v, int g)
{
    v.a = gsum(v.a, g);
    v.b = gsum(v.b, g);
    v.c = gsum(v.c, g);
    v.d = gsum(v.d, g);
}

// Left-looking block LDU of node record x (FactorizeGraphA, pull form):
//   D_j  = A_jj - sum_{i in R(j)} W_ji U_ij
//   W_kj = A_kj - sum_i W_ki U_ij,  V_jk = A_jk - sum_i W_ji U_ik  (k in S(j))
//   stored: LU[s] <- (W_kj, U_jk = D_j^-1 V_jk), and with STORE_D the D
//   section <- D_j^-1 (needed only by later solves with these factors).
// With FWD, also the forward substitution and normalisation of the rhs:
//   y_j = D_j^-1 (b_j - sum_{i in R(j)} W_ji y_i).
// Loads are issued in batches so that the chain of dependent requests per
// node stays short: the record's dependants first (diagonal inputs, rhs,
// the first two destinations' slot records, the first R indices), then R(j)
// four entries per lane at a time, then two destinations per step with both
// update chains in flight together.  Every load is in bounds: absent items
// read entry 0 and are masked out.
// SYM: a symmetric matrix (eq. 2 blockwise): only the lower blocks take
// updates and U_jk = D_j^-1 W_kj^T.
template <class SRC, bool FWD, bool STORE_D, bool SYM = false>
__device__ __forceinline__ void factor_node(const DevSym& S, const SRC& src, const NodeRec& rec,
                                            int lane, int g, const View& w, int64_t lu,
                                            const View& wr, int64_t rhs, int* s_bad)
{
    const int4 n0 = rec.a;
    const int4 n1 = rec.b;
    const int j = n0.x, bus = n0.y;
    const int r1 = n0.w, s1 = n1.y;
    const typename SRC::DiagIn din = src.diag_in(j, bus, n1.z);
    double2 bj = make_double2(0.0, 0.0);
    if (FWD) bj = wr.v2(rhs + 2 * (int64_t)j);
    int s = n1.x + lane;
    int sc = s < s1 ? s : 0, sc2 = s + g < s1 ? s + g : 0;
    int4 sa = S.slot_info[2 * sc], sb = S.slot_info[2 * sc + 1];
    int4 sa2 = S.slot_info[2 * sc2], sb2 = S.slot_info[2 * sc2 + 1];
    int2 e[4];
    int r = n0.z + lane;
#pragma unroll
    for (int k = 0; k < 4; ++k) e[k] = S.rl[r + k * g < r1 ? r + k * g : 0];
    Blk ds = bzero();
    double z0 = 0.0, z1 = 0.0;
    for (; r < r1; r += 4 * g) {
        Blk wv[4], uv[4];
        double2 yi[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            wv[k] = w.blk(lu + 8 * (int64_t)e[k].y);
            uv[k] = w.blk(lu + 8 * (int64_t)e[k].y + 4);
            if (FWD) yi[k] = wr.v2(rhs + 2 * (int64_t)e[k].x);
        }
        const int rn = r + 4 * g;
#pragma unroll
        for (int k = 0; k < 4; ++k) e[k] = S.rl[rn + k * g < r1 ? rn + k * g : 0];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (r + k * g < r1) {
                bmadd(ds, wv[k], uv[k]);
                if (FWD) mvadd(z0, z1, wv[k], yi[k].x, yi[k].y);
            }
        }
    }
    if (g > 1) {
        gsum_blk(ds, g);
        if (FWD) {
            z0 = gsum(z0, g);
            z1 = gsum(z1, g);
        }
    }
    const Blk Ajj = src.diag_of(din);
    bool ok;
    const Blk Di = binv({Ajj.a - ds.a, Ajj.b - ds.b, Ajj.c - ds.c, Ajj.d - ds.d}, ok);
    for (; s < s1; s += 2 * g) {
        const int s2 = s + g;
        const bool two = s2 < s1;
        const typename SRC::OffIn o1 = src.off_in(s, sa.y, sa.z, sa.w);
        const typename SRC::OffIn o2 = src.off_in(two ? s2 : s, sa2.y, sa2.z, sa2.w);
        const int u0 = sb.x, u1 = sb.y, v0 = two ? sb2.x : 0, v1 = two ? sb2.y : 0;
        const int2 p = upd_at(S.upd, u0, u1), q = upd_at(S.upd, v0, v1);
        const int sn = s + 2 * g;
        sc = sn < s1 ? sn : 0;
        sc2 = sn + g < s1 ? sn + g : 0;
        sa = S.slot_info[2 * sc];
        sb = S.slot_info[2 * sc + 1];
        sa2 = S.slot_info[2 * sc2];
        sb2 = S.slot_info[2 * sc2 + 1];
        Blk Wk, Vk, Wk2, Vk2;
        src.off_of(din, o1, Wk, Vk);
        src.off_of(din, o2, Wk2, Vk2);
        apply_updates2<SYM>(S.upd, u0, u1, v0, v1, p, q, w, lu, Wk, Vk, Wk2, Vk2);
        w.put(lu + 8 * (int64_t)s, Wk);
        w.put(lu + 8 * (int64_t)s + 4, bmul(Di, SYM ? btrans(Wk) : Vk));
        if (two) {
            w.put(lu + 8 * (int64_t)s2, Wk2);
            w.put(lu + 8 * (int64_t)s2 + 4, bmul(Di, SYM ? btrans(Wk2) : Vk2));
        }
    }
    if (lane == 0) {
        if (!ok) *s_bad = 1;
        if (STORE_D) w.put(4 * (int64_t)j, Di);
        if (FWD) {
            double y0 = 0.0, y1 = 0.0;
            mvadd(y0, y1, Di, bj.x - z0, bj.y - z1);
            wr.put2(rhs + 2 * (int64_t)j, make_double2(y0, y1));
        }
    }
}

// Local slot of clique pair (a, b), a < b: the clique's slots are numbered
// node by node, node a owning KC - a - 1 of them.
__device__ __forceinline__ int clique_slot(int c0, int KC, int a, int b)
{
    return c0 + a * (KC - 1) - (a * (a - 1)) / 2 + (b - a - 1);
}

// The LDS tail of the factorisation.
// Phase A (all threads, no ordering): every tail diagonal, rhs entry and
//   slot takes the updates of descendants outside the tail (global memory).
// Phase B: the tail levels below the clique, in order, in LDS.
// Phase C: clique entries take the updates of tail nodes below the clique.
// Phase D: the clique as a dense block, right-looking: at pivot a every
//   thread forms D_a^-1 and y_a itself, then the trailing blocks (k, l) are
//   updated in parallel, A_kl -= W_ka D_a^-1 V_al, with one barrier per
//   pivot; row a is normalised (U_al = D_a^-1 V_al) during pivot a + 1,
//   when nobody reads it any more.
// WRITE stores the tail's factors to global memory.
template <class SRC, bool FWD, bool WRITE>
__device__ void tail_factor(const DevSym& S, const SRC& src, const View& w, int64_t lu,
                            const View& wr, int64_t rhs, int* s_bad)
{
    const int K = S.tail_nodes, TS = S.tail_slots, KC = S.tail_clique;
    const int nT = S.nlev - S.tail_level;
    double* sLU = pf_smem;             // TS x 8: W, then V -> U
    double* sD = pf_smem + 8 * TS;     // K x 4: accumulated pivot, then D^-1
    double* sy = sD + 4 * K;           // K x 2: accumulated rhs, then y
    for (int it = threadIdx.x; it < K + TS; it += blockDim.x) {
        if (it < K) {
            const int4 t0 = S.t_node[3 * it];
            const int4 t1 = S.t_node[3 * it + 1];
            Blk acc = src.diag(t0.x, t0.y, t0.z);
            double z0 = 0.0, z1 = 0.0;
            if (FWD) {
                const double2 b = wr.v2(rhs + 2 * (int64_t)t0.x);
                z0 = b.x;
                z1 = b.y;
            }
            for (int r = t1.y; r < t1.z; ++r) {
                const int2 e = S.t_rl[r];
                const Blk wv = w.blk(lu + 8 * (int64_t)e.y);
                bmsub(acc, wv, w.blk(lu + 8 * (int64_t)e.y + 4));
                if (FWD) {
                    const double2 yi = wr.v2(rhs + 2 * (int64_t)e.x);
                    z0 = fma(-wv.a, yi.x, fma(-wv.b, yi.y, z0));
                    z1 = fma(-wv.c, yi.x, fma(-wv.d, yi.y, z1));
                }
            }
            bstore(sD + 4 * it, acc);
            sy[2 * it] = z0;
            sy[2 * it + 1] = z1;
        } else {
            const int t = it - K;
            const int4 a = S.t_slot[3 * t];
            const int4 b = S.t_slot[3 * t + 1];
            const int4 c = S.t_slot[3 * t + 2];
            Blk Wk, Vk;
            src.off(a.x, c.x, a.z, a.w, b.x, Wk, Vk);
            apply_updates(S.t_upd, b.y, b.z, w, lu, Wk, Vk);
            bstore(sLU + 8 * t, Wk);
            bstore(sLU + 8 * t + 4, Vk);
        }
    }
    __syncthreads();
    for_tail_range(S, 0, nT - KC, true, [&](int jl, int lane, int g) {
        const int4 t0 = S.t_node[3 * jl];
        const int4 t1 = S.t_node[3 * jl + 1];
        Blk ds = bzero();
        double z0 = 0.0, z1 = 0.0;
        for (int r = t1.z + lane; r < t1.w; r += g) {
            const int2 e = S.t_rl[r];
            const Blk wv = bload(sLU + 8 * e.y);
            bmadd(ds, wv, bload(sLU + 8 * e.y + 4));
            if (FWD) mvadd(z0, z1, wv, sy[2 * e.x], sy[2 * e.x + 1]);
        }
        if (g > 1) {
            gsum_blk(ds, g);
            if (FWD) {
                z0 = gsum(z0, g);
                z1 = gsum(z1, g);
            }
        }
        const Blk A = bload(sD + 4 * jl);
        bool ok;
        const Blk Di = binv({A.a - ds.a, A.b - ds.b, A.c - ds.c, A.d - ds.d}, ok);
        for (int t = t0.w + lane; t < t1.x; t += g) {
            const int4 b = S.t_slot[3 * t + 1];
            Blk Wk = bload(sLU + 8 * t), Vk = bload(sLU + 8 * t + 4);
            apply_updates_lds(S.t_upd, b.z, b.w, sLU, Wk, Vk);
            bstore(sLU + 8 * t, Wk);
            bstore(sLU + 8 * t + 4, bmul(Di, Vk));
        }
        if (lane == 0) {
            if (!ok) *s_bad = 1;
            bstore(sD + 4 * jl, Di);
            if (FWD) {
                double y0 = 0.0, y1 = 0.0;
                mvadd(y0, y1, Di, sy[2 * jl] - z0, sy[2 * jl + 1] - z1);
                sy[2 * jl] = y0;
                sy[2 * jl + 1] = y1;
            }
        }
    });
    if (KC > 0) {
        const int kf = K - KC;
        const int c0 = S.t_node[3 * kf].w;  // first local slot of the clique
        // phase C: clique diagonals, rhs and slots take the tail updates from below
        for (int it = threadIdx.x; it < KC + (TS - c0); it += blockDim.x) {
            if (it < KC) {
                // the packed local R list, below-clique part (its prefix)
                const int jl = kf + it;
                const int4 t1 = S.t_node[3 * jl + 1];
                const int4 t2 = S.t_node[3 * jl + 2];
                const int nR = t2.x - t1.z;
                Blk acc = bload(sD + 4 * jl);
                double z0 = sy[2 * jl], z1 = sy[2 * jl + 1];
                uint4 q = S.t_pk[nR > 0 ? t2.y : 0];
                for (int k = 0; k < nR; k += 4) {
                    const uint4 qn = S.t_pk[k + 4 < nR ? t2.y + (k >> 2) + 1 : 0];
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        if (k + c < nR) {
                            const uint32_t v = pk_word(q, c);
                            const int il = v & 0xffff, sl = v >> 16;
                            const Blk wv = bload(sLU + 8 * sl);
                            bmsub(acc, wv, bload(sLU + 8 * sl + 4));
                            if (FWD) {
                                z0 = fma(-wv.a, sy[2 * il], fma(-wv.b, sy[2 * il + 1], z0));
                                z1 = fma(-wv.c, sy[2 * il], fma(-wv.d, sy[2 * il + 1], z1));
                            }
                        }
                    }
                    q = qn;
                }
                bstore(sD + 4 * jl, acc);
                sy[2 * jl] = z0;
                sy[2 * jl + 1] = z1;
            } else {
                // the packed local pair list, below-clique part (its prefix)
                const int t = c0 + (it - KC);
                const int4 b = S.t_slot[3 * t + 1];
                const int4 c = S.t_slot[3 * t + 2];
                Blk Wk = bload(sLU + 8 * t), Vk = bload(sLU + 8 * t + 4);
                Blk W2 = bzero(), V2 = bzero();
                apply_packed2_lds(S.t_pk, c.w, c.z - b.z, 0, 0, sLU, Wk, Vk, W2, V2);
                bstore(sLU + 8 * t, Wk);
                bstore(sLU + 8 * t + 4, Vk);
            }
        }
        __syncthreads();
        // phase D: dense right-looking over the clique's pivots.  Pivots with a
        // large trailing block use every thread, one barrier each; the last
        // ones (at most two updates per lane of one wavefront) run on the
        // first wavefront alone, without workgroup barriers.
        Blk Dprev = bzero();
        double yp0 = 0.0, yp1 = 0.0;
        auto pivot = [&](int a, int stride) {
            const int m = KC - 1 - a;  // trailing size
            Blk Di = bzero();
            double ya0 = 0.0, ya1 = 0.0;
            if (a < KC) {
                const int ja = kf + a;
                bool ok;
                Di = binv(bload(sD + 4 * ja), ok);
                if (!ok && threadIdx.x == 0) *s_bad = 1;
                if (FWD) mvadd(ya0, ya1, Di, sy[2 * ja], sy[2 * ja + 1]);
            }
            const int nupd = (a < KC) ? m * m : 0;
            const int nnorm = (a > 0) ? (KC - a) + 1 : 0;  // row a-1 slots + its pivot
            for (int it = threadIdx.x; it < nupd + nnorm; it += stride) {
                if (it < nupd) {
                    const unsigned q = (unsigned)it / (unsigned)m;
                    const int k = a + 1 + (int)q, l = a + 1 + (it - (int)q * m);
                    const Blk Wka = bload(sLU + 8 * clique_slot(c0, KC, a, k));
                    const Blk Ual = bmul(Di, bload(sLU + 8 * clique_slot(c0, KC, a, l) + 4));
                    const int jk = kf + k;
                    if (k == l) {
                        Blk d = bload(sD + 4 * jk);
                        bmsub(d, Wka, Ual);
                        bstore(sD + 4 * jk, d);
                        if (FWD) {
                            sy[2 * jk] = fma(-Wka.a, ya0, fma(-Wka.b, ya1, sy[2 * jk]));
                            sy[2 * jk + 1] = fma(-Wka.c, ya0, fma(-Wka.d, ya1, sy[2 * jk + 1]));
                        }
                    } else if (k > l) {
                        double* p = sLU + 8 * clique_slot(c0, KC, l, k);
                        Blk v = bload(p);
                        bmsub(v, Wka, Ual);
                        bstore(p, v);
                    } else {
                        double* p = sLU + 8 * clique_slot(c0, KC, k, l) + 4;
                        Blk v = bload(p);
                        bmsub(v, Wka, Ual);
                        bstore(p, v);
                    }
                } else {
                    const int r = it - nupd;  // normalise row a-1
                    const int jp = kf + a - 1;
                    if (r < KC - a) {
                        double* p = sLU + 8 * clique_slot(c0, KC, a - 1, a + r) + 4;
                        bstore(p, bmul(Dprev, bload(p)));
                    } else {
                        bstore(sD + 4 * jp, Dprev);
                        if (FWD) {
                            sy[2 * jp] = yp0;
                            sy[2 * jp + 1] = yp1;
                        }
                    }
                }
            }
            Dprev = Di;
            yp0 = ya0;
            yp1 = ya1;
        };
        int a = 0;
        for (; a <= KC && (KC - 1 - a) * (KC - 1 - a) > 2 * kWave; ++a) {
            pivot(a, blockDim.x);
            __syncthreads();
        }
        if (threadIdx.x < kWave) {
            for (int b = a; b <= KC; ++b) {
                pivot(b, kWave);
                wave_sync();
            }
        }
        __syncthreads();
    }
    if (WRITE) {
        for (int t = threadIdx.x; t < TS; t += blockDim.x) {
            const int s = S.t_slot[3 * t].x;
            w.put(lu + 8 * (int64_t)s, bload(sLU + 8 * t));
            w.put(lu + 8 * (int64_t)s + 4, bload(sLU + 8 * t + 4));
        }
        for (int jl = threadIdx.x; jl < K; jl += blockDim.x) {
            const int j = S.t_node[3 * jl].x;
            w.put(4 * (int64_t)j, bload(sD + 4 * jl));
            if (FWD) wr.put2(rhs + 2 * (int64_t)j, make_double2(sy[2 * jl], sy[2 * jl + 1]));
        }
        __syncthreads();
    }
}

// Newton step of one bus: theta -= dtheta, |V| -= d|V| (PQ), new e + jf;
// the record's first 32 bytes (e, f, |V|, theta) are rewritten in one store.
__device__ __forceinline__ void apply_step_to(const View& w, int64_t rec, const Blk& r, bool pv,
                                              double x0, double x1)
{
    const double va = r.d - x0;
    const double vm = pv ? r.c : r.c - x1;
    double sn, cs;
    sincos(va, &sn, &cs);
    w.put(rec, {vm * cs, vm * sn, vm, va});
}

__device__ __forceinline__ void apply_step(const View& w, int64_t rec, bool pv, double x0,
                                           double x1)
{
    apply_step_to(w, rec, w.blk(rec), pv, x0, x1);
}

// Backward substitution of the tail from LDS: x_j = y_j - sum U_jk x_k.  The
// clique goes first, on the first wavefront alone, column-oriented: once x_a
// is final, y_k -= U_ka x_a for every clique node k below a.  The x of the
// tail nodes are written to the rhs (for the levels below) and, with UPDATE,
// applied to the bus records in one parallel pass at the end, so that no
// level waits for a bus-record load.  With xs (the solution vector in LDS by
// position, over the tail's own LDS; at most four tail nodes per thread) the
// x go there instead of the rhs: each thread takes its x into registers,
// and writes them after a barrier.
template <bool UPDATE>
__device__ void tail_backward(const DevSym& S, const View& w, int64_t rhs, int64_t bus_off,
                              PvMask type, double2* xs)
{
    const int K = S.tail_nodes, TS = S.tail_slots, KC = S.tail_clique;
    const int nT = S.nlev - S.tail_level;
    const double* sLU = pf_smem;
    double* sy = pf_smem + 8 * TS + 4 * K;
    if (KC > 0) {
        if (threadIdx.x < kWave) {
            const int kf = K - KC;
            const int c0 = S.t_node[3 * kf].w;
            for (int a = KC - 1; a > 0; --a) {
                const int ja = kf + a;
                const double x0 = sy[2 * ja], x1 = sy[2 * ja + 1];
                for (int k = threadIdx.x; k < a; k += kWave) {
                    const int jk = kf + k;
                    const Blk U = bload(sLU + 8 * clique_slot(c0, KC, k, a) + 4);
                    sy[2 * jk] = fma(-U.a, x0, fma(-U.b, x1, sy[2 * jk]));
                    sy[2 * jk + 1] = fma(-U.c, x0, fma(-U.d, x1, sy[2 * jk + 1]));
                }
                wave_sync();
            }
        }
        __syncthreads();
    }
    for_tail_range(S, 0, nT - KC, false, [&](int jl, int lane, int g) {
        const int4 t0 = S.t_node[3 * jl];
        const int4 t1 = S.t_node[3 * jl + 1];
        double a0 = 0.0, a1 = 0.0;
        for (int t = t0.w + lane; t < t1.x; t += g) {
            const int kl = S.t_slot[3 * t].y;
            mvadd(a0, a1, bload(sLU + 8 * t + 4), sy[2 * kl], sy[2 * kl + 1]);
        }
        if (g > 1) {
            a0 = gsum(a0, g);
            a1 = gsum(a1, g);
        }
        if (lane == 0) {
            sy[2 * jl] -= a0;
            sy[2 * jl + 1] -= a1;
        }
    });
    if (xs) {
        double2 xr[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int jl = threadIdx.x + r * blockDim.x;
            xr[r] = jl < K ? make_double2(sy[2 * jl], sy[2 * jl + 1]) : make_double2(0.0, 0.0);
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int jl = threadIdx.x + r * blockDim.x;
            if (jl < K) {
                const int4 t0 = S.t_node[3 * jl];
                xs[t0.x] = xr[r];
                if (UPDATE)
                    apply_step(w, bus_off + 8 * (int64_t)t0.y, type(t0.y), xr[r].x, xr[r].y);
            }
        }
    } else {
        for (int jl = threadIdx.x; jl < K; jl += blockDim.x) {
            const int4 t0 = S.t_node[3 * jl];
            const double x0 = sy[2 * jl], x1 = sy[2 * jl + 1];
            w.put2(rhs + 2 * (int64_t)t0.x, make_double2(x0, x1));
            if (UPDATE) apply_step(w, bus_off + 8 * (int64_t)t0.y, type(t0.y), x0, x1);
        }
    }
    __syncthreads();
}

// Backward substitution of node record x: x_j = y_j - sum_{k in S(j)} U_jk x_k,
// four slots per lane at a time (next indices in flight), the node's own
// rhs entry and bus record requested first.
template <bool UPDATE>
__device__ __forceinline__ void back_node(const DevSym& S, const NodeRec& rec, int lane, int g,
                                          const View& w, int64_t lu, const View& wb,
                                          int64_t rhs, int64_t bus_off, PvMask type,
                                          double2* xs)
{
    const int4 n0 = rec.a;
    const int4 n1 = rec.b;
    const int s1 = n1.y;
    const double2 y = wb.v2(rhs + 2 * (int64_t)n0.x);
    const int64_t brec = bus_off + 8 * (int64_t)n0.y;
    Blk br = bzero();
    bool pv = false;
    if (UPDATE) {
        br = wb.blk(brec);
        pv = type(n0.y);
    }
    int s = n1.x + lane;
    int kk[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) kk[k] = S.Li[s + k * g < s1 ? s + k * g : 0];
    double a0 = 0.0, a1 = 0.0;
    for (; s < s1; s += 4 * g) {
        Blk u[4];
        double2 xk[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int sk = s + k * g < s1 ? s + k * g : 0;
            u[k] = w.blk(lu + 8 * (int64_t)sk + 4);
            xk[k] = xs ? xs[kk[k]] : wb.v2(rhs + 2 * (int64_t)kk[k]);
        }
        const int sn = s + 4 * g;
#pragma unroll
        for (int k = 0; k < 4; ++k) kk[k] = S.Li[sn + k * g < s1 ? sn + k * g : 0];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (s + k * g < s1) mvadd(a0, a1, u[k], xk[k].x, xk[k].y);
    }
    if (g > 1) {
        a0 = gsum(a0, g);
        a1 = gsum(a1, g);
    }
    if (lane == 0) {
        const double x0 = y.x - a0, x1 = y.y - a1;
        if (xs) xs[n0.x] = make_double2(x0, x1);
        else wb.put2(rhs + 2 * (int64_t)n0.x, make_double2(x0, x1));
        if (UPDATE) apply_step_to(wb, brec, br, pv, x0, x1);
    }
}

// Max over the workgroup with a NaN flag; every thread gets the result.
__device__ double block_max(double v, int nan, int& any_nan)
{
    __shared__ double s_v[kMaxThreads / 64 + 1];
    __shared__ int s_n[kMaxThreads / 64 + 1];
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    nan = __any(nan);
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_v[wv] = v;
        s_n[wv] = nan;
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
    int interleave;
    int B;
    int32_t* iters;
    double* norm;
    int32_t* status;
};

struct CaseDesc {
    DevSym sym;
    int64_t bus_off, br_off, y_off, ws_off;
};

// Mismatch pass of one case: P + jQ into the bus records and F = calculated
// - scheduled (F_Q = 0 at PV buses) into the rhs in position order, divided
// by |V| with SCALE (the fast decoupled right-hand sides); the thread's max
// |F| and NaN flag accumulate into mx and nan.  Buses are taken in bus
// order, two per thread per step, so that the admittance rows, row pointers,
// positions and scheduled injections of a wavefront are adjacent in memory;
// all loads of both buses are issued before either is summed.
template <bool SCALE, class EF>
__device__ __forceinline__ void mismatch_pass(const DevSym& S, const double* yv, const EF& ef,
                                              const View& wb, const Off& o, const PvMask& pvm,
                                              const double* Psp, const double* Qsp, double& mx,
                                              int& nan)
{
    const int bd = blockDim.x;
    for (int i = threadIdx.x; i < S.n; i += 2 * bd) {
        const int i2 = i + bd;
        const bool two = i2 < S.n;
        const int ic = two ? i2 : i;
        const int pc = S.pos[i], pd = S.pos[ic];
        const int qc0 = S.yptr[i], qc1 = S.yptr[i + 1];
        const int qd0 = S.yptr[ic], qd1 = S.yptr[ic + 1];
        const double spc = Psp[i], sqc = Qsp[i], spd = Psp[ic], sqd = Qsp[ic];
        const int64_t rc = o.BUS + 8 * (int64_t)i, rd = o.BUS + 8 * (int64_t)ic;
        Blk vc, vd;  // e, f, |V| (|V| only with SCALE)
        if (SCALE) {
            vc = wb.blk(rc);
            vd = wb.blk(rd);
        } else {
            ef.get(i, vc.a, vc.b);
            ef.get(ic, vd.a, vd.b);
            vc.c = vd.c = 1.0;
        }
        const bool pvc = pvm(i), pvd = pvm(ic);
        int kc[4], kd[4];
        RowHead hc, hd;
        row_head_idx<EF>(S, yv, qc0, qc1, kc, hc);
        row_head_idx<EF>(S, yv, qd0, qd1, kd, hd);
        row_head_v(ef, kc, hc);
        row_head_v(ef, kd, hd);
        double p, q, p2, q2;
        row_finish(S, yv, ef, qc0, qc1, hc, vc.a, vc.b, p, q);
        row_finish(S, yv, ef, qd0, qd1, hd, vd.a, vd.b, p2, q2);
        if (pc >= 0) {  // the slack is not a position
            const double fp = p - spc, fq = pvc ? 0.0 : q - sqc;
            wb.put2(rc + 4, make_double2(p, q));
            wb.put2(o.RHS + 2 * (int64_t)pc,
                    SCALE ? make_double2(fp / vc.c, fq / vc.c) : make_double2(fp, fq));
            nan |= (fp != fp) | (fq != fq);
            mx = fmax(mx, fmax(fabs(fp), fabs(fq)));
        }
        if (two && pd >= 0) {
            const double fp2 = p2 - spd, fq2 = pvd ? 0.0 : q2 - sqd;
            wb.put2(rd + 4, make_double2(p2, q2));
            wb.put2(o.RHS + 2 * (int64_t)pd, SCALE ? make_double2(fp2 / vd.c, fq2 / vd.c)
                                                     : make_double2(fp2, fq2));
            nan |= (fp2 != fp2) | (fq2 != fq2);
            mx = fmax(mx, fmax(fabs(fp2), fabs(fq2)));
        }
    }
}

// The whole Newton-Raphson loop of one case, run by one workgroup.  The
// case's voltages and injections are copied into its bus records first and
// the solution copied back at the end.
__device__ void newton_case(const DevSym& S, const double* yv, const int8_t* type,
                            const double* Psp, const double* Qsp, double* Vm, double* Va,
                            const View& w, const View& wb, double tol, int max_iter,
                            int flags, int32_t* o_iters, double* o_norm, int32_t* o_status)
{
    __shared__ int s_bad;
    const Off o = ws_off(S);
    for (int i = threadIdx.x; i < S.n; i += blockDim.x) {
        double sn, cs;
        const double vm = Vm[i], va = Va[i];
        sincos(va, &sn, &cs);
        wb.put(o.BUS + 8 * (int64_t)i, {vm * cs, vm * sn, vm, va});
    }
    pv_fill(S, type);
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    const PvMask pvm{pv_words(S)};
    // the global levels of the factorisation sweep read neighbours' (e, f)
    // from the LDS copy the mismatch pass just made (the tail reuses that LDS
    // afterwards and reads them from the bus records)
    const SrcState src{yv, pvm, wb, o.BUS,
                       S.ef_lds ? reinterpret_cast<const double2*>(pf_smem) : nullptr};
    // the backward sweep keeps x in that LDS too (free again once the tail's
    // backward substitution has read its values)
    double2* const xs = (S.ef_lds && S.tail_nodes <= 4 * (int)blockDim.x)
                            ? reinterpret_cast<double2*>(pf_smem)
                            : nullptr;
    const EFView ef{wb, o.BUS};
    const bool tail = S.tail_nodes > 0;
    int it = 0, st = ST_NOT_CONVERGED;
    double nrm = 0.0;
    for (;;) {
        double mx = 0.0;
        int nan = 0;
        if (S.ef_lds) {
            // every bus's (e, f) into LDS (free until the tail), so that the
            // admittance rows' voltages are LDS reads
            const EFLds efl{reinterpret_cast<double2*>(pf_smem)};
            for (int i = threadIdx.x; i < S.n; i += blockDim.x)
                efl.s[i] = wb.v2(o.BUS + 8 * (int64_t)i);
            __syncthreads();
            mismatch_pass<false>(S, yv, efl, wb, o, pvm, Psp, Qsp, mx, nan);
        } else {
            mismatch_pass<false>(S, yv, ef, wb, o, pvm, Psp, Qsp, mx, nan);
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
        if (it >= max_iter) {
            st = ST_NOT_CONVERGED;
            break;
        }
        for_nodes(S, 0, S.tail_level, true, [&](int, const NodeRec& r, int lane, int g) {
            factor_node<SrcState, true, false>(S, src, r, lane, g, w, o.LU, wb, o.RHS, &s_bad);
        });
        if (tail) tail_factor<SrcState, true, false>(S, src, w, o.LU, wb, o.RHS, &s_bad);
        if (s_bad) {
            st = ST_ZERO_PIVOT;
            break;
        }
        if (tail) tail_backward<true>(S, wb, o.RHS, o.BUS, pvm, xs);
        for_nodes(S, 0, S.tail_level, false, [&](int, const NodeRec& r, int lane, int g) {
            back_node<true>(S, r, lane, g, w, o.LU, wb, o.RHS, o.BUS, pvm, xs);
        });
        ++it;
    }
    if ((flags & PF_NEWTON_KEEP_FACTORS) && st == ST_OK) {
        for_nodes(S, 0, S.tail_level, true, [&](int, const NodeRec& r, int lane, int g) {
            factor_node<SrcState, false, true>(S, src, r, lane, g, w, o.LU, wb, o.RHS, &s_bad);
        });
        if (tail) tail_factor<SrcState, false, true>(S, src, w, o.LU, wb, o.RHS, &s_bad);
        if (s_bad) st = ST_ZERO_PIVOT;
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
        int2 e[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) e[k] = S.rl[r + k * g < r1 ? r + k * g : 0];
        double z = 0.0;
        for (; r < r1; r += 4 * g) {
            double w[4], y[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                w[k] = sl[e[k].y].x;
                y[k] = fd_x<VL>(xv, wb, rhs, comp, e[k].x);
            }
            const int rn = r + 4 * g;
#pragma unroll
            for (int k = 0; k < 4; ++k) e[k] = S.rl[rn + k * g < r1 ? rn + k * g : 0];
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
        int s = rec.b.x + lane;
        int kk[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) kk[k] = S.Li[s + k * g < s1 ? s + k * g : 0];
        double a = 0.0;
        for (; s < s1; s += 4 * g) {
            double u[4], x[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                u[k] = sl[s + k * g < s1 ? s + k * g : 0].y;
                x[k] = fd_x<VL>(xv, wb, rhs, comp, kk[k]);
            }
            const int sn = s + 4 * g;
#pragma unroll
            for (int k = 0; k < 4; ++k) kk[k] = S.Li[sn + k * g < s1 ? sn + k * g : 0];
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
                                                        int32_t* status)
{
    __shared__ int s_bad;
    const int c = case_of_block(blockIdx.x, C, B);
    if (c < 0) return;
    const View w = case_view(vals, vals_stride, C, c);
    const int64_t lu = S.lu_off;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    const SrcLoadT<SYM> src{w, lu};
    for_nodes(S, 0, S.tail_level, true, [&](int, const NodeRec& r, int lane, int g) {
        factor_node<SrcLoadT<SYM>, false, true, SYM>(S, src, r, lane, g, w, lu, w, 0, &s_bad);
    });
    if (S.tail_nodes > 0) tail_factor<SrcLoadT<SYM>, false, true>(S, src, w, lu, w, 0, &s_bad);
    __syncthreads();
    if (threadIdx.x == 0 && status) status[c] = s_bad ? ST_ZERO_PIVOT : ST_OK;
}

// transpose = 0: y_j = D_j^-1 (b_j - sum_{i in R(j)} W_ji y_i)  (levels up),
//                x_j = y_j - sum_{k in S(j)} U_jk x_k            (levels down).
// transpose = 1: p_j = g_j - sum_{i in R(j)} U_ij^T p_i           (levels up),
//                l_j = D_j^-T (p_j - sum_{k in S(j)} W_kj^T l_k)  (levels down).
// A node's g lanes take its list entries in strides of g, four per lane per
// step with the step's blocks and x values requested together; absent
// entries of a step re-read the node's first entry (in bounds whenever the
// list is not empty) and add nothing.  LDSX keeps the case's whole vector
// in LDS (nn x 16 bytes) for the two sweeps.
template <bool TRANS, bool LDSX>
__global__ __launch_bounds__(kLevelThreads) void k_solve(DevSym S, const double* vals,
                                                       int64_t vals_stride, int C, int B,
                                                       double* rhs, int64_t rhs_stride)
{
    const int c = case_of_block(blockIdx.x, C, B);
    if (c < 0) return;
    const View w = case_view(const_cast<double*>(vals), vals_stride, C, c);
    const int64_t lu = S.lu_off;
    double2* xg = reinterpret_cast<double2*>(rhs + c * rhs_stride);
    double2* x2 = LDSX ? reinterpret_cast<double2*>(pf_smem) : xg;
    if (LDSX) {
        for (int p = threadIdx.x; p < S.nn; p += blockDim.x) x2[p] = xg[p];
        __syncthreads();
    }
    for_nodes(S, 0, S.nlev, true, [&](int, const NodeRec& rec, int lane, int g) {
        const int j = rec.a.x, r0 = rec.a.z, r1 = rec.a.w;
        double z0 = 0.0, z1 = 0.0;
        for (int base = r0 + lane; base < r1; base += 4 * g) {
            int2 e[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int r = base + k * g;
                e[k] = S.rl[r < r1 ? r : r0];
            }
            Blk M[4];
            double2 xv[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                M[k] = w.blk(lu + 8 * (int64_t)e[k].y + (TRANS ? 4 : 0));
                xv[k] = x2[e[k].x];
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
            z0 = gsum(z0, g);
            z1 = gsum(z1, g);
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
    for_nodes(S, 0, S.nlev, false, [&](int, const NodeRec& rec, int lane, int g) {
        const int j = rec.a.x, s0 = rec.b.x, s1 = rec.b.y;
        double a0 = 0.0, a1 = 0.0;
        for (int base = s0 + lane; base < s1; base += 4 * g) {
            int sk[4], kk[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int s = base + k * g;
                sk[k] = s < s1 ? s : s0;
                kk[k] = S.Li[sk[k]];
            }
            Blk M[4];
            double2 xv[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                M[k] = w.blk(lu + 8 * (int64_t)sk[k] + (TRANS ? 0 : 4));
                xv[k] = x2[kk[k]];
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
            a0 = gsum(a0, g);
            a1 = gsum(a1, g);
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
    if (LDSX)
        for (int p = threadIdx.x; p < S.nn; p += blockDim.x) xg[p] = x2[p];
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
        newton_case(S, a.yval + cd.y_off, a.type + cd.bus_off, a.Psp + cd.bus_off,
                    a.Qsp + cd.bus_off, a.Vm + cd.bus_off, a.Va + cd.bus_off, w, wb, a.tol,
                    a.max_iter, a.flags, a.iters ? a.iters + c : nullptr,
                    a.norm ? a.norm + c : nullptr, a.status ? a.status + c : nullptr);
    } else {
        const int c = case_of_block(blockIdx.x, a.interleave, a.B);
        if (c < 0) return;
        const View w = case_view(a.ws, a.ws_stride, a.interleave, c);
        const View wb = case_bus_view(a.ws, a.ws_stride, a.interleave, c, Sarg.vals_doubles);
        newton_case(Sarg, a.yval + c * a.y_stride, a.type + c * a.type_stride,
                    a.Psp + c * a.inj_stride, a.Qsp + c * a.inj_stride, a.Vm + c * a.v_stride,
                    a.Va + c * a.v_stride, w, wb, a.tol, a.max_iter, a.flags,
                    a.iters ? a.iters + c : nullptr, a.norm ? a.norm + c : nullptr,
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
__device__ __forceinline__ double adj_branch(const DevSym& S, int fb, int tb,
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
    return -acc;
}

// mode 1 (x shared by the cases): one workgroup per 64 branches, its waves
// split the cases and combine them in a fixed order, so no atomics are
// needed and the sum is reproducible.  mode 0: one thread per (case, branch).
__global__ void k_adj_branch(DevSym S, const int32_t* __restrict__ from,
                             const int32_t* __restrict__ to, int B, const double* lam,
                             int64_t lam_stride, const int8_t* type, int64_t type_stride,
                             const double* Vm, const double* Va, int64_t v_stride,
                             const double* r, const double* x, int64_t branch_stride,
                             double* gx, int mode)
{
    if (mode == 1) {
        __shared__ double part[16][64];
        const int e = blockIdx.x * 64 + (threadIdx.x & 63);
        const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
        double acc = 0.0;
        if (e < S.m) {
            const int fb = from[e], tb = to[e];
            for (int c = wv; c < B; c += nw)
                acc += adj_branch(S, fb, tb, lam + c * lam_stride, type + c * type_stride,
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
            adj_branch(S, from[e], to[e], lam + c * lam_stride, type + c * type_stride,
                       Vm + c * v_stride, Va + c * v_stride, r[c * branch_stride + e],
                       x[c * branch_stride + e]);
    }
}


// Fast decoupled matrices of B cases: B' then B'' (fd_mat doubles each) in
// the scalar filled layout, lower and upper values equal.
__global__ void k_fd_matrices(DevSym S, const double* __restrict__ r,
                              const double* __restrict__ x, const double* __restrict__ b,
                              int64_t bstride, const int8_t* __restrict__ type,
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
    m1[p] = fd_entry<false>(S, S.ydiag[p], true, rc, xc, bc);
    m2[p] = pvj ? 1.0 : fd_entry<true>(S, S.ydiag[p], true, rc, xc, bc);
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


// ---------------------------------------------------------------------------
// WLS state estimation (Sec. IV names it among the applications run on the
// same machinery; the formulation is the textbook one).  Gauss-Newton steps
// G dx = H^T W (z - h(x)), G = H^T W H, on 2x2 blocks per bus (unknowns
// theta, |V|); G is assembled into the filled layout of its own analysis
// and factored and solved by the level-scheduled kernels.
// ---------------------------------------------------------------------------
struct SeDev {
    int M, ref;           // measurements; reference bus (theta fixed)
    const int8_t* kind;   // 1 |V|, 2 P, 3 Q (bus), 4 P_ft, 5 Q_ft (branch)
    const int32_t* loc;   // bus or branch
    const int32_t* sup;   // M+1: first partial of each measurement
    const int32_t* blk;   // nn + nnz_l + 1 (gain analysis): contribution ranges
    const int4* ent;      // (m, partial of the row bus, partial of the column bus, 0)
    const int32_t* rptr;  // nn + 1: rhs contribution ranges per position
    const int2* rent;     // (m, partial of the bus)
    const int32_t* from;  // network branch ends
    const int32_t* to;
};

// The estimator's workspace for a batch of B cases.  Per-measurement data
// are case-minor (entry e of case c at e * B + c) so that a wavefront whose
// lanes are 64 cases of one measurement or one position reads them
// coalesced; the gain matrix is in the filled layout of its analysis in
// interleaved groups of C cases, the rhs plain per case.
struct SeWs {
    int B, C;
    double* vals;   // gain matrix, groups of C cases, stride vs
    int64_t vs;
    double* rhs;    // [B][rs]: H^T W r, then the step
    int64_t rs;
    double* y;      // admittance values, [B][ys] (ys = 0: one copy for all)
    int64_t ys;
    double2* st;    // [n][B] x 2: (e, f), (|V|, theta)
    double2* par;   // [P][B]: (dh/dtheta_b, dh/d|V|_b)
    double* res;    // [M][B]: z - h
};

// Case-minor state of every bus: (e, f, |V|, theta) from the caller's |V|, theta.
__global__ __launch_bounds__(64) void k_se_state(int n, SeWs X, const double* __restrict__ Vm,
                                                 const double* __restrict__ Va, int64_t vstride,
                                                 const int32_t* __restrict__ status)
{
    const int i = blockIdx.x;
    const int c = blockIdx.y * 64 + threadIdx.x;
    if (c >= X.B || status[c] >= 0) return;
    const double vm = Vm[c * vstride + i], va = Va[c * vstride + i];
    double sn, cs;
    sincos(va, &sn, &cs);
    double2* s = X.st + 2 * ((int64_t)i * X.B + c);
    s[0] = make_double2(vm * cs, vm * sn);
    s[1] = make_double2(vm, va);
}

// Measurement values (residual z - h) and partials d h / d(theta_b, |V_b|)
// for every bus b of the support, in the support's order; one measurement
// per workgroup, lanes over cases.
__global__ __launch_bounds__(64) void k_se_eval(DevSym N, SeDev E, SeWs X,
                                                const double* __restrict__ r,
                                                const double* __restrict__ x,
                                                const double* __restrict__ b, int64_t bstride,
                                                const double* __restrict__ z, int64_t zstride,
                                                const int32_t* __restrict__ status)
{
    const int mi = blockIdx.x;
    const int c = blockIdx.y * 64 + threadIdx.x;
    if (c >= X.B || status[c] >= 0) return;
    const int B = X.B;
    auto ef = [&](int bus) { return X.st[2 * ((int64_t)bus * B + c)]; };
    auto vm = [&](int bus) { return X.st[2 * ((int64_t)bus * B + c) + 1].x; };
    auto par = [&](int p) -> double2& { return X.par[(int64_t)p * B + c]; };
    const int kind = E.kind[mi], loc = E.loc[mi], p0 = E.sup[mi];
    double h = 0.0;
    if (kind == 1) {
        h = vm(loc);
        par(p0) = make_double2(0.0, 1.0);
    } else if (kind == 2 || kind == 3) {
        const double2* yv = reinterpret_cast<const double2*>(X.y + c * X.ys);
        const int i = loc, q0 = N.yptr[i], q1 = N.yptr[i + 1];
        const double2 vi = ef(i);
        const double ei = vi.x, fi = vi.y;
        double ir = 0.0, ii = 0.0, gd = 0.0, bd = 0.0;
        for (int q = q0; q < q1; ++q) {
            const int k = N.ycol[q];
            const double2 y = yv[q];
            const double2 vk = ef(k);
            ir = fma(y.x, vk.x, fma(-y.y, vk.y, ir));
            ii = fma(y.x, vk.y, fma(y.y, vk.x, ii));
            if (k == i) {
                gd = y.x;
                bd = y.y;
            }
        }
        const double P = ei * ir + fi * ii, Q = fi * ir - ei * ii;
        h = kind == 2 ? P : Q;
        for (int q = q0; q < q1; ++q) {
            const int k = N.ycol[q];
            Blk J;
            if (k == i) {
                J = jac_diag(gd, bd, P, Q, vm(i), false);
            } else {
                const double2 y = yv[q];
                const double2 vk = ef(k);
                J = jac_off(y.x, y.y, ei, fi, vk.x, vk.y, vm(k), false, false);
            }
            par(p0 + (q - q0)) = kind == 2 ? make_double2(J.a, J.b) : make_double2(J.c, J.d);
        }
    } else {
        // S_f = |V_f|^2 conj(y_ff) + V_f conj(c), c = y_ft V_t, y_ff = y + jb/2,
        // y_ft = -y:  dS/dtheta_f = j V_f conj(c) = -dS/dtheta_t,
        // dS/d|V_f| = 2|V_f| conj(y_ff) + (V_f/|V_f|) conj(c),
        // dS/d|V_t| = V_f conj(c) / |V_t|
        const int e = loc, fb = E.from[e], tb = E.to[e];
        const double rr = r[c * bstride + e], xx = x[c * bstride + e];
        const double hb = b[c * bstride + e] / 2.0;
        const double den = rr * rr + xx * xx;
        const double yg = rr / den, yb = -xx / den;
        const double2 Vf = ef(fb), Vt = ef(tb);
        const double vf = vm(fb), vt = vm(tb);
        const double ef_ = Vf.x, ff = Vf.y, et = Vt.x, ft = Vt.y;
        const double cr = -(yg * et - yb * ft), ci = -(yg * ft + yb * et);  // c = -y V_t
        const double ar = ef_ * cr + ff * ci, ai = ff * cr - ef_ * ci;     // V_f conj(c)
        const double Sr = vf * vf * yg + ar, Si = -vf * vf * (yb + hb) + ai;
        // partials as complex numbers (re, im)
        const double dthf_r = -ai, dthf_i = ar;                  // j a
        const double dvf_r = 2 * vf * yg + ar / vf, dvf_i = -2 * vf * (yb + hb) + ai / vf;
        const double dvt_r = ar / vt, dvt_i = ai / vt;
        const bool Pm = kind == 4;
        h = Pm ? Sr : Si;
        const double tf = Pm ? dthf_r : dthf_i, vff = Pm ? dvf_r : dvf_i;
        const double tt = -tf, vtt = Pm ? dvt_r : dvt_i;
        const int lo = fb < tb ? 0 : 1;  // the support is (min, max) of the ends
        par(p0 + lo) = make_double2(tf, vff);
        par(p0 + 1 - lo) = make_double2(tt, vtt);
    }
    X.res[(int64_t)mi * B + c] = z[c * zstride + mi] - h;
}

// G = H^T W H and H^T W (z - h) into the filled layout of the gain analysis:
// one position per workgroup (its diagonal block, the blocks of its slots and
// its rhs entry), lanes over cases.  The reference bus's angle row and
// column become identity.
__global__ __launch_bounds__(64) void k_se_assemble(DevSym S, SeDev E, SeWs X,
                                                    const double* __restrict__ wt,
                                                    int64_t wstride,
                                                    const int32_t* __restrict__ status)
{
    const int j = blockIdx.x;
    const int c = blockIdx.y * 64 + threadIdx.x;
    if (c >= X.B || status[c] >= 0) return;
    const int B = X.B;
    const View w = case_view(X.vals, X.vs, X.C, c);
    const double* wc = wt + c * wstride;
    auto par = [&](int p) { return X.par[(int64_t)p * B + c]; };
    auto block = [&](int q) {
        Blk g = bzero();
        for (int t = E.blk[q]; t < E.blk[q + 1]; ++t) {
            const int4 en = E.ent[t];
            const double wm = wc[en.x];
            const double2 a = par(en.y), bb = par(en.z);
            g.a = fma(wm * a.x, bb.x, g.a);
            g.b = fma(wm * a.x, bb.y, g.b);
            g.c = fma(wm * a.y, bb.x, g.c);
            g.d = fma(wm * a.y, bb.y, g.d);
        }
        return g;
    };
    const bool refj = S.perm[j] == E.ref;
    Blk D = block(j);
    double r0 = 0.0, r1 = 0.0;
    for (int t = E.rptr[j]; t < E.rptr[j + 1]; ++t) {
        const int2 en = E.rent[t];
        const double v = wc[en.x] * X.res[(int64_t)en.x * B + c];
        const double2 a = par(en.y);
        r0 = fma(v, a.x, r0);
        r1 = fma(v, a.y, r1);
    }
    if (refj) {
        D = {1.0, 0.0, 0.0, D.d};
        r0 = 0.0;
    }
    w.put(4 * (int64_t)j, D);
    reinterpret_cast<double2*>(X.rhs + c * X.rs)[j] = make_double2(r0, r1);
    for (int s = S.Lp[j]; s < S.Lp[j + 1]; ++s) {
        Blk L = block(S.nn + s);  // block (k, j), k = Li[s]
        const bool refk = S.perm[S.Li[s]] == E.ref;
        if (refj) {  // angle column of the reference
            L.a = 0.0;
            L.c = 0.0;
        }
        if (refk) {  // angle row of the reference
            L.a = 0.0;
            L.b = 0.0;
        }
        w.put(S.lu_off + 8 * (int64_t)s, L);
        w.put(S.lu_off + 8 * (int64_t)s + 4, btrans(L));
    }
}

// x += dx at every bus (angle fixed at the reference); per case the max
// |dx| decides: converged (< tol), not converged after max_iter steps, or
// non-finite.  Cases already decided are left alone.
__global__ __launch_bounds__(kLevelThreads) void k_se_update(
    DevSym S, SeDev E, SeWs X, double* Vm, double* Va, int64_t vstride, double tol, int it,
    int max_iter, int32_t* iters, double* norm, int32_t* status)
{
    const int c = blockIdx.x;
    if (status[c] >= 0) return;
    const double2* dx = reinterpret_cast<const double2*>(X.rhs + c * X.rs);
    double* vm = Vm + c * vstride;
    double* va = Va + c * vstride;
    double mx = 0.0;
    int nan = 0;
    for (int p = threadIdx.x; p < S.nn; p += blockDim.x) {
        const int bus = S.perm[p];
        const double2 d = dx[p];
        const double dt = bus == E.ref ? 0.0 : d.x;
        va[bus] += dt;
        vm[bus] += d.y;
        nan |= (d.x != d.x) | (d.y != d.y);
        mx = fmax(mx, fmax(fabs(dt), fabs(d.y)));
    }
    int any_nan = 0;
    const double nrm = block_max(mx, nan, any_nan);
    if (threadIdx.x == 0) {
        norm[c] = nrm;
        iters[c] = it + 1;
        if (any_nan || !isfinite(nrm)) status[c] = ST_NONFINITE;
        else if (nrm < tol) status[c] = ST_OK;
        else if (it + 1 >= max_iter) status[c] = ST_NOT_CONVERGED;
    }
}

__global__ void k_se_start(int B, int32_t* iters, double* norm, int32_t* status)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= B) return;
    iters[c] = 0;
    norm[c] = 0.0;
    status[c] = -1;
}

// ===========================================================================
// C ABI
// ===========================================================================
struct pf_symbolic_s {
    HostSym h;
    const int32_t* d_from = nullptr;  // device copies of the branch ends
    const int32_t* d_to = nullptr;
};

struct pf_multi_s {
    std::vector<pf_symbolic> syms;
    std::vector<int64_t> bus_off, br_off, y_off, ws_off;
    std::vector<int32_t> order;
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

// Workgroup size of the level-scheduled kernels: the symbolic's setting, or
// by batch size so that a small batch still brings 16 waves to its CUs.
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

// Dynamic LDS of the Newton kernel: the tail and the (e, f) copy share the
// front, the PV mask follows the larger of the two.
int newton_lds(const HostSym& h)
{
    return std::max(h.tail_lds, h.ef_lds) + (int)pv_mask_bytes(h.n);
}

int launch_threads(const HostSym& h, int B)
{
    if (h.threads > 0) return h.threads;
    return B <= 512 ? 512 : 256;
}

int grid_blocks(int B, int C);
void allow_big_lds();

// The level-scheduled factorisation of B matrices (sym: symmetric ones).
void factor_launch(const HostSym& h, int B, double* vals, int64_t stride, int C,
                   int32_t* status, hipStream_t st, bool sym)
{
    allow_big_lds();
    if (sym)
        hipLaunchKernelGGL(k_factor<true>, dim3(grid_blocks(B, C)), dim3(launch_threads(h, B)),
                           h.tail_lds, st, h.dev, vals, stride, C, B, status);
    else
        hipLaunchKernelGGL(k_factor<false>, dim3(grid_blocks(B, C)), dim3(launch_threads(h, B)),
                           h.tail_lds, st, h.dev, vals, stride, C, B, status);
}

// Blocks for B cases in groups of C placed one XCD round apart.
int grid_blocks(int B, int C)
{
    if (C <= 1) return B;
    const int span = 8 * C;
    return ((B + span - 1) / span) * span;
}

bool valid_interleave(int C) { return C == 1 || C == 2 || C == 4 || C == 8; }

// Interleave pf_newton uses for B cases: the symbolic's setting, reduced so
// that a group never outnumbers the batch (a lone case stays contiguous).
int newton_interleave(const HostSym& h, int B)
{
    int C = h.interleave;
    while (C > 1 && C > B) C >>= 1;
    return C;
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
    const void* kernels[] = {reinterpret_cast<const void*>(&k_newton<false>),
                             reinterpret_cast<const void*>(&k_newton<true>),
                             reinterpret_cast<const void*>(&k_factor<false>),
                             reinterpret_cast<const void*>(&k_factor<true>),
                             reinterpret_cast<const void*>(&k_solve<false, true>),
                             reinterpret_cast<const void*>(&k_solve<true, true>),
                             reinterpret_cast<const void*>(&k_fdpf)};
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


// ---- WLS state estimation: host plan -----------------------------------------
struct pf_se_s {
    pf_symbolic_s net, gain;
    int n = 0, m = 0, M = 0, ref = 0;
    int64_t P = 0;
    std::vector<int8_t> kind;
    std::vector<int32_t> loc, sup, blk, ent, rptr, rent;
    size_t net_bytes = 0, gain_bytes = 0, arr_bytes = 0;
    SeDev dev{};
    bool uploaded = false;
    int64_t vs = 0, rs = 0, ys = 0, ws = 0;  // workspace sections per case (doubles)
};

namespace {

int64_t round8(int64_t v) { return (v + 7) & ~(int64_t)7; }

int se_plan(pf_se_s& E, int n, int m, const int32_t* from, const int32_t* to, int slack, int M,
            const int8_t* kind, const int32_t* loc, std::string& msg)
{
    int rc = pf::analyze(n, m, from, to, slack, PF_ORDER_MINDEG, E.net.h, msg);
    if (rc != PF_OK) return rc;
    const HostSym& N = E.net.h;
    E.n = n;
    E.m = m;
    E.M = M;
    E.ref = slack;
    E.kind.assign(kind, kind + M);
    E.loc.assign(loc, loc + M);
    // supports (ascending buses; an injection's is its admittance row)
    E.sup.assign(M + 1, 0);
    std::vector<int32_t> sb;
    for (int i = 0; i < M; ++i) {
        const int k = kind[i], l = loc[i];
        if (k == 1 || k == 2 || k == 3) {
            if (l < 0 || l >= n) {
                msg = "pf_se_analyze: bus measurement location out of range";
                return PF_E_INVALID;
            }
            if (k == 1) sb.push_back(l);
            else
                for (int q = N.yptr[l]; q < N.yptr[l + 1]; ++q) sb.push_back(N.ycol[q]);
        } else if (k == 4 || k == 5) {
            if (l < 0 || l >= m) {
                msg = "pf_se_analyze: branch measurement location out of range";
                return PF_E_INVALID;
            }
            sb.push_back(std::min(from[l], to[l]));
            sb.push_back(std::max(from[l], to[l]));
        } else {
            msg = "pf_se_analyze: unknown measurement kind";
            return PF_E_INVALID;
        }
        E.sup[i + 1] = (int32_t)sb.size();
    }
    E.P = (int64_t)sb.size();
    // gain-matrix graph: buses sharing a measurement, plus a dummy bus n
    // joined to bus 0 as the analysis' slack, so every bus stays a node
    std::vector<int64_t> keys;
    for (int i = 0; i < M; ++i)
        for (int a = E.sup[i]; a < E.sup[i + 1]; ++a)
            for (int b = a + 1; b < E.sup[i + 1]; ++b)
                if (sb[a] != sb[b])
                    keys.push_back((int64_t)std::min(sb[a], sb[b]) * (n + 1) +
                                   std::max(sb[a], sb[b]));
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    std::vector<int32_t> gf(keys.size() + 1), gt(keys.size() + 1);
    for (size_t e = 0; e < keys.size(); ++e) {
        gf[e] = (int32_t)(keys[e] / (n + 1));
        gt[e] = (int32_t)(keys[e] % (n + 1));
    }
    gf[keys.size()] = n;
    gt[keys.size()] = 0;
    rc = pf::analyze(n + 1, (int)gf.size(), gf.data(), gt.data(), n, PF_ORDER_MINDEG, E.gain.h,
                     msg);
    if (rc == PF_E_DISCONNECTED) msg = "pf_se_analyze: the measurements leave buses unobservable";
    if (rc != PF_OK) return rc;
    const HostSym& G = E.gain.h;
    const int nn = G.nn;
    const int64_t nz = (int64_t)G.Li.size();
    auto slot = [&](int p, int q) -> int64_t {  // q in S(p)
        const auto b = G.Li.begin() + G.Lp[p], e = G.Li.begin() + G.Lp[p + 1];
        const auto it = std::lower_bound(b, e, q);
        return (it != e && *it == q) ? it - G.Li.begin() : -1;
    };
    // contribution lists: counting pass, then fill
    std::vector<int32_t> cnt(nn + nz + 1, 0), rc_cnt(nn + 1, 0);
    auto visit = [&](bool fill, std::vector<int32_t>& pos_b, std::vector<int32_t>& pos_r) {
        for (int i = 0; i < M; ++i) {
            const int a0 = E.sup[i], a1 = E.sup[i + 1];
            for (int a = a0; a < a1; ++a) {
                const int pa = G.pos[sb[a]];
                if (fill) {
                    const int t = pos_r[pa]++;
                    E.rent[2 * t] = i;
                    E.rent[2 * t + 1] = a;
                } else {
                    ++rc_cnt[pa + 1];
                }
                for (int bq = a0; bq < a1; ++bq) {
                    const int pb = G.pos[sb[bq]];
                    int64_t q = -1;
                    if (pa == pb && a == bq) q = pa;
                    else if (pa > pb) q = nn + slot(pb, pa);
                    if (q < 0) continue;
                    if (fill) {
                        const int t = pos_b[q]++;
                        E.ent[4 * t] = i;
                        E.ent[4 * t + 1] = a;
                        E.ent[4 * t + 2] = bq;
                    } else {
                        ++cnt[q + 1];
                    }
                }
            }
        }
    };
    std::vector<int32_t> dummy;
    visit(false, dummy, dummy);
    for (size_t q = 0; q + 1 < cnt.size(); ++q) cnt[q + 1] += cnt[q];
    for (size_t q = 0; q + 1 < rc_cnt.size(); ++q) rc_cnt[q + 1] += rc_cnt[q];
    E.blk = cnt;
    E.rptr = rc_cnt;
    E.ent.assign(4 * (size_t)cnt.back(), 0);
    E.rent.assign(2 * (size_t)rc_cnt.back(), 0);
    std::vector<int32_t> pb(cnt.begin(), cnt.end() - 1), pr(rc_cnt.begin(), rc_cnt.end() - 1);
    visit(true, pb, pr);
    // workspace per case: gain values | rhs | admittances | state (4 per bus) |
    // partials | residuals (the last three case-minor across the batch)
    E.vs = round8(G.vals_doubles());
    E.rs = round8(2 * (int64_t)nn);
    E.ys = round8(2 * (int64_t)N.ycol.size());
    E.ws = round8(E.vs + E.rs + E.ys + 4 * (int64_t)n + 2 * E.P + M);
    return PF_OK;
}

size_t se_arr_bytes(const pf_se_s& E)
{
    auto a = [](size_t b) { return (std::max<size_t>(b, 4) + 255) & ~(size_t)255; };
    return a(E.kind.size()) + a(4 * E.loc.size()) + a(4 * E.sup.size()) + a(4 * E.blk.size()) +
           a(4 * E.ent.size()) + a(4 * E.rptr.size()) + a(4 * E.rent.size());
}

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
    info->lu_offset = h.lu_off();
    info->fd_mat_doubles = 2 * h.fd_mat();
    info->fd_ws_doubles = h.fd_ws_doubles();
    info->ws_doubles = h.ws_doubles();
    info->dev_bytes = h.dev_bytes();
    info->tail_levels = (int32_t)h.level_ptr.size() - 1 - h.tail_level;
    info->tail_nodes = h.tail_nodes;
    info->tail_lds_bytes = h.tail_lds;
    info->tail_clique = h.tail_clique;
    info->ws_interleave = h.interleave;
    info->threads = h.threads;
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

int pf_symbolic_set_launch(pf_symbolic s, int threads, int64_t tail_lds_budget, int interleave)
{
    if (!s) return fail(PF_E_INVALID, "pf_symbolic_set_launch: NULL symbolic");
    if (!valid_interleave(interleave))
        return fail(PF_E_INVALID, "pf_symbolic_set_launch: interleave must be 1, 2, 4 or 8");
    s->h.interleave = interleave;
    if (threads != 0 && threads != 64 && threads != 128 && threads != 256 && threads != 512)
        return fail(PF_E_INVALID, "pf_symbolic_set_launch: threads must be 0, 64, 128, 256 or 512");
    if (tail_lds_budget < 0 || tail_lds_budget > 158 * 1024)
        return fail(PF_E_INVALID, "pf_symbolic_set_launch: tail budget must be 0..161792 bytes");
    s->h.threads = threads;
    if (tail_lds_budget != s->h.tail_budget) {
        s->h.tail_budget = tail_lds_budget;
        pf::build_tail(s->h, tail_lds_budget);
        s->h.uploaded = false;  // device copy is stale: upload again
    }
    return PF_OK;
}

int pf_newton_interleave(const pf_symbolic s, int B)
{
    if (!s || B < 0) return fail(PF_E_INVALID, "pf_newton_interleave: bad arguments"), -1;
    return newton_interleave(s->h, B);
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
    d.lu_off = h.lu_off();
    d.fd_lu = h.fd_lu();
    d.fd_mat = h.fd_mat();
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
    d.level_ptr = put(h.level_ptr);
    d.level_nodes = put(h.level_nodes);
    d.level_g = put(h.level_g);
    d.node_info = reinterpret_cast<const int4*>(put(h.node_info));
    d.slot_info = reinterpret_cast<const int4*>(put(h.slot_info));
    d.rl = reinterpret_cast<const int2*>(put(h.rl));
    d.upd = reinterpret_cast<const int2*>(put(h.upd));
    d.tail_level = h.tail_level;
    d.tail_nodes = h.tail_nodes;
    d.tail_slots = h.tail_slots;
    d.tail_lds = h.tail_lds;
    d.tail_clique = h.tail_clique;
    d.ef_lds = 0;
    d.t_node = reinterpret_cast<const int4*>(put(h.t_node));
    d.t_slot = reinterpret_cast<const int4*>(put(h.t_slot));
    d.t_rl = reinterpret_cast<const int2*>(put(h.t_rl));
    d.t_upd = reinterpret_cast<const int2*>(put(h.t_upd));
    d.t_lptr = put(h.t_lptr);
    d.t_pk = reinterpret_cast<const uint4*>(put(h.t_pk));
    s->d_from = put(h.from);
    s->d_to = put(h.to);
    if (off > info.dev_bytes) return fail(PF_E_WORKSPACE, "pf_symbolic_upload: size mismatch");
    {
        int dev = 0, lds_max = 0;
        h.ef_lds = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) ==
                hipSuccess) {
            if (h.tail_lds + pv_mask_bytes(h.n) + 2048 > lds_max)
                return fail(PF_E_WORKSPACE, "pf_symbolic_upload: LDS tail larger than the "
                                            "device's LDS; lower it with pf_symbolic_set_launch");
            const int64_t efb = 16 * (int64_t)h.n;
            if (efb + pv_mask_bytes(h.n) + 2048 <= lds_max) h.ef_lds = (int32_t)efb;
        } else {
            (void)hipGetLastError();
        }
        d.ef_lds = h.ef_lds;
    }
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
                int64_t v_stride, double* d_vals, int64_t vals_stride, int vals_interleave,
                void* stream)
{
    if (!ready(s, "pf_jacobian")) return PF_E_INVALID;
    if (B < 0 || B > 65535 || !d_yval || !d_type || !d_Vm || !d_Va || !d_vals ||
        !valid_interleave(vals_interleave) || (vals_stride & 7))
        return fail(PF_E_INVALID, "pf_jacobian: bad arguments");
    if (B > 1 && vals_stride < s->h.vals_doubles())
        return fail(PF_E_WORKSPACE, "pf_jacobian: vals_stride < vals_doubles");
    if (B == 0 || s->h.nn == 0) return PF_OK;
    dim3 grid((s->h.nn + 255) / 256, B);
    hipLaunchKernelGGL(k_jacobian, grid, dim3(256), 0, as_stream(stream), s->h.dev, d_yval,
                       y_stride, d_type, type_stride, d_Vm, d_Va, v_stride, d_vals, vals_stride,
                       vals_interleave);
    return launch_check("pf_jacobian");
}

int pf_factor(const pf_symbolic s, int B, double* d_vals, int64_t vals_stride,
              int vals_interleave, int32_t* d_status, void* stream)
{
    if (!ready(s, "pf_factor")) return PF_E_INVALID;
    if (B < 0 || !d_vals || !valid_interleave(vals_interleave) || (vals_stride & 7))
        return fail(PF_E_INVALID, "pf_factor: bad arguments");
    if (B > 1 && vals_stride < s->h.vals_doubles())
        return fail(PF_E_WORKSPACE, "pf_factor: vals_stride < vals_doubles");
    if (B == 0) return PF_OK;
    factor_launch(s->h, B, d_vals, vals_stride, vals_interleave, d_status, as_stream(stream),
                  false);
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
    if (B > 1 && v_stride < s->h.n)
        return fail(PF_E_WORKSPACE, "pf_newton: v_stride too small");
    if (ws_stride < s->h.ws_doubles() || (ws_stride & 7))
        return fail(PF_E_WORKSPACE, "pf_newton: ws_stride must be >= ws_doubles, a multiple of 8");
    if (reinterpret_cast<uintptr_t>(d_ws) & 15)
        return fail(PF_E_WORKSPACE, "pf_newton: workspace must be 16-byte aligned");
    if (B == 0) return PF_OK;
    const int C = newton_interleave(s->h, B);
    NewtonArgs a{d_yval, y_stride, d_type, type_stride, d_Psp, d_Qsp, inj_stride, d_Vm, d_Va,
                 v_stride, d_ws, ws_stride, tol, max_iter, flags, C, B, d_iters, d_norm,
                 d_status};
    allow_big_lds();
    hipLaunchKernelGGL(k_newton<false>, dim3(grid_blocks(B, C)), dim3(launch_threads(s->h, B)),
                       newton_lds(s->h), as_stream(stream), s->h.dev, (const CaseDesc*)nullptr,
                       (const int32_t*)nullptr, a);
    return launch_check("pf_newton");
}

int pf_fdpf_matrices(const pf_symbolic s, int B, const double* d_r, const double* d_x,
                     const double* d_b, int64_t branch_stride, const int8_t* d_type,
                     int64_t type_stride, double* d_mat, int64_t mat_stride, void* stream)
{
    if (!ready(s, "pf_fdpf_matrices")) return PF_E_INVALID;
    if (B < 0 || B > 65535 || !d_r || !d_x || !d_b || !d_type || !d_mat || (mat_stride & 7))
        return fail(PF_E_INVALID, "pf_fdpf_matrices: bad arguments");
    if (reinterpret_cast<uintptr_t>(d_mat) & 15)
        return fail(PF_E_WORKSPACE, "pf_fdpf_matrices: d_mat must be 16-byte aligned");
    if (B > 1 && mat_stride < 2 * s->h.fd_mat())
        return fail(PF_E_WORKSPACE, "pf_fdpf_matrices: mat_stride < fd_mat_doubles");
    if (B == 0) return PF_OK;
    dim3 grid((unsigned)((s->h.fd_lu() + 255) / 256), B);
    hipLaunchKernelGGL(k_fd_matrices, grid, dim3(256), 0, as_stream(stream), s->h.dev, d_r, d_x,
                       d_b, branch_stride, d_type, type_stride, d_mat, mat_stride);
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
    if (ws_stride < s->h.fd_ws_doubles() || (ws_stride & 7))
        return fail(PF_E_WORKSPACE,
                    "pf_fdpf: ws_stride must be >= fd_ws_doubles, a multiple of 8");
    if ((reinterpret_cast<uintptr_t>(d_ws) & 15) || (reinterpret_cast<uintptr_t>(d_mat) & 15))
        return fail(PF_E_WORKSPACE, "pf_fdpf: d_ws and d_mat must be 16-byte aligned");
    if (B == 0) return PF_OK;
    NewtonArgs a{d_yval, y_stride, d_type, type_stride, d_Psp, d_Qsp, inj_stride, d_Vm, d_Va,
                 v_stride, d_ws, ws_stride, tol, max_iter, 0, 1, B, d_iters, d_norm, d_status};
    allow_big_lds();
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
    if (B == 0 || s->h.m == 0) return PF_OK;
    dim3 grid((s->h.m + 255) / 256, B);
    hipLaunchKernelGGL(k_branch_flows, grid, dim3(256), 0, as_stream(stream), s->h.m, s->d_from,
                       s->d_to, d_r, d_x, d_b, branch_stride, d_Vm, d_Va, v_stride, d_Pft, d_Qft,
                       d_Ptf, d_Qtf, out_stride);
    return launch_check("pf_branch_flows");
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
        const dim3 grid(gx_mode == 1 ? (s->h.m + 63) / 64 : (s->h.m + 255) / 256,
                        gx_mode == 1 ? 1 : B);
        const dim3 block(gx_mode == 1 ? 1024 : 256);
        hipLaunchKernelGGL(k_adj_branch, grid, block, 0, as_stream(stream), s->h.dev,
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
                 flags, 1, (int)p->syms.size(), d_iters, d_norm, d_status};
    DevSym none{};
    int lds = 0, threads = 0;
    for (auto* sy : p->syms) {
        lds = std::max(lds, newton_lds(sy->h));
        threads = std::max(threads, sy->h.threads);
    }
    if (threads == 0) threads = (p->syms.size() <= 512) ? 512 : 256;
    allow_big_lds();
    hipLaunchKernelGGL(k_newton<true>, dim3(p->syms.size()), dim3(threads), lds,
                       as_stream(stream), none, p->d_desc, p->d_order, a);
    return launch_check("pf_newton_multi");
}

void pf_multi_destroy(pf_multi p) { delete p; }

int pf_se_analyze(int n, int m, const int32_t* from, const int32_t* to, int slack, int M,
                  const int8_t* kind, const int32_t* loc, pf_se* out)
{
    if (!out) return fail(PF_E_INVALID, "pf_se_analyze: out is NULL");
    *out = nullptr;
    if (M <= 0 || !kind || !loc) return fail(PF_E_INVALID, "pf_se_analyze: no measurements");
    try {
        pf_se s = new pf_se_s();
        std::string msg;
        const int rc = se_plan(*s, n, m, from, to, slack, M, kind, loc, msg);
        if (rc != PF_OK) {
            delete s;
            return fail(rc, msg);
        }
        *out = s;
        g_err.clear();
        return PF_OK;
    } catch (const std::exception& ex) {
        return fail(PF_E_INVALID, std::string("pf_se_analyze: ") + ex.what());
    }
}

int pf_se_info(const pf_se s, pf_se_dims* info)
{
    if (!s || !info) return fail(PF_E_INVALID, "pf_se_info: NULL argument");
    pf_info ni, gi;
    pf_symbolic_info(const_cast<pf_symbolic>(&s->net), &ni);
    pf_symbolic_info(const_cast<pf_symbolic>(&s->gain), &gi);
    info->n = s->n;
    info->m = s->m;
    info->measurements = s->M;
    info->partials = s->P;
    info->gain_nnz_l = gi.nnz_l;
    info->gain_levels = gi.nlevels;
    info->contributions = (int64_t)s->ent.size() / 4;
    info->ws_doubles = s->ws;
    info->dev_bytes = ni.dev_bytes + gi.dev_bytes + se_arr_bytes(*s);
    return PF_OK;
}

int pf_se_set_launch(pf_se s, int threads, int64_t tail_lds_budget)
{
    if (!s) return fail(PF_E_INVALID, "pf_se_set_launch: NULL argument");
    const int rc = pf_symbolic_set_launch(&s->gain, threads, tail_lds_budget, 1);
    if (rc == PF_OK) s->uploaded = false;
    return rc;
}

int pf_se_upload(pf_se s, void* d_buf, size_t bytes, void* stream)
{
    if (!s || !d_buf) return fail(PF_E_INVALID, "pf_se_upload: NULL argument");
    pf_se_dims info;
    pf_se_info(s, &info);
    if (bytes < info.dev_bytes)
        return fail(PF_E_WORKSPACE, "pf_se_upload: buffer smaller than dev_bytes");
    if (reinterpret_cast<uintptr_t>(d_buf) & 255)
        return fail(PF_E_WORKSPACE, "pf_se_upload: buffer not 256-byte aligned");
    pf_info ni, gi;
    pf_symbolic_info(&s->net, &ni);
    pf_symbolic_info(&s->gain, &gi);
    char* base = static_cast<char*>(d_buf);
    int rc = pf_symbolic_upload(&s->net, base, ni.dev_bytes, stream);
    if (rc) return rc;
    rc = pf_symbolic_upload(&s->gain, base + ni.dev_bytes, gi.dev_bytes, stream);
    if (rc) return rc;
    char* arr = base + ni.dev_bytes + gi.dev_bytes;
    std::vector<char> stage(se_arr_bytes(*s), 0);
    size_t off = 0;
    auto put = [&](const void* p, size_t nb) -> const void* {
        if (nb) std::memcpy(stage.data() + off, p, nb);
        const void* d = arr + off;
        off += (std::max<size_t>(nb, 4) + 255) & ~(size_t)255;
        return d;
    };
    SeDev d{};
    d.M = s->M;
    d.ref = s->ref;
    d.kind = static_cast<const int8_t*>(put(s->kind.data(), s->kind.size()));
    d.loc = static_cast<const int32_t*>(put(s->loc.data(), 4 * s->loc.size()));
    d.sup = static_cast<const int32_t*>(put(s->sup.data(), 4 * s->sup.size()));
    d.blk = static_cast<const int32_t*>(put(s->blk.data(), 4 * s->blk.size()));
    d.ent = static_cast<const int4*>(put(s->ent.data(), 4 * s->ent.size()));
    d.rptr = static_cast<const int32_t*>(put(s->rptr.data(), 4 * s->rptr.size()));
    d.rent = static_cast<const int2*>(put(s->rent.data(), 4 * s->rent.size()));
    d.from = s->net.d_from;
    d.to = s->net.d_to;
    rc = hip_check(hipMemcpyAsync(arr, stage.data(), off, hipMemcpyHostToDevice,
                                  as_stream(stream)),
                   "pf_se_upload: hipMemcpyAsync");
    if (rc) return rc;
    rc = hip_check(hipStreamSynchronize(as_stream(stream)), "pf_se_upload: sync");
    if (rc) return rc;
    s->dev = d;
    s->uploaded = true;
    return PF_OK;
}

// Cases per interleaved group of the gain matrix.
constexpr int kSeGroup = 4;

int pf_se_estimate(const pf_se s, int B, const double* d_r, const double* d_x,
                   const double* d_b, int64_t branch_stride, const double* d_z,
                   int64_t z_stride, const double* d_w, int64_t w_stride, double* d_Vm,
                   double* d_Va, int64_t v_stride, double tol, int max_iter, double* d_ws,
                   int64_t ws_size, int32_t* d_iters, double* d_norm, int32_t* d_status,
                   void* stream)
{
    if (!s || !s->uploaded) return fail(PF_E_INVALID, "pf_se_estimate: not uploaded");
    if (B < 0 || B > 65535 || max_iter < 1 || !(tol >= 0.0) || !d_r || !d_x || !d_b || !d_z ||
        !d_w || !d_Vm || !d_Va || !d_ws || !d_iters || !d_norm || !d_status || z_stride < 0 ||
        w_stride < 0 || branch_stride < 0)
        return fail(PF_E_INVALID, "pf_se_estimate: bad arguments");
    if (B > 1 && (v_stride < s->n || (z_stride != 0 && z_stride < s->M) ||
                  (w_stride != 0 && w_stride < s->M) ||
                  (branch_stride != 0 && branch_stride < s->m)))
        return fail(PF_E_WORKSPACE, "pf_se_estimate: stride too small");
    const int Bg = (B + kSeGroup - 1) / kSeGroup * kSeGroup;
    if (ws_size < (int64_t)Bg * s->ws || (reinterpret_cast<uintptr_t>(d_ws) & 15))
        return fail(PF_E_WORKSPACE, "pf_se_estimate: d_ws must hold ceil(B/4)*4 * ws_doubles "
                                    "doubles and be 16-byte aligned");
    if (B == 0) return PF_OK;
    hipStream_t st = as_stream(stream);
    const HostSym& G = s->gain.h;
    const int yb = branch_stride ? B : 1;  // admittance copies
    SeWs X;
    X.B = B;
    X.C = kSeGroup;
    X.vals = d_ws;
    X.vs = s->vs;
    X.rhs = X.vals + (int64_t)Bg * s->vs;
    X.rs = s->rs;
    X.y = X.rhs + (int64_t)B * s->rs;
    X.ys = branch_stride ? s->ys : 0;
    X.st = reinterpret_cast<double2*>(X.y + (int64_t)yb * s->ys);
    X.par = X.st + 2 * (int64_t)s->n * B;
    X.res = reinterpret_cast<double*>(X.par + s->P * B);
    hipLaunchKernelGGL(k_se_start, dim3((B + 255) / 256), dim3(256), 0, st, B, d_iters, d_norm,
                       d_status);
    int rc = launch_check("pf_se_estimate: start");
    if (rc) return rc;
    rc = pf_build_ybus(&s->net, yb, d_r, d_x, d_b, branch_stride, X.y, s->ys, stream);
    if (rc) return rc;
    const unsigned cg = (unsigned)((B + 63) / 64);
    std::vector<int32_t> host(B);
    for (int it = 0; it < max_iter; ++it) {
        hipLaunchKernelGGL(k_se_state, dim3(s->n, cg), dim3(64), 0, st, s->n, X, d_Vm, d_Va,
                           v_stride, d_status);
        if ((rc = launch_check("pf_se_estimate: state"))) return rc;
        hipLaunchKernelGGL(k_se_eval, dim3(s->M, cg), dim3(64), 0, st, s->net.h.dev, s->dev, X,
                           d_r, d_x, d_b, branch_stride, d_z, z_stride, d_status);
        if ((rc = launch_check("pf_se_estimate: eval"))) return rc;
        hipLaunchKernelGGL(k_se_assemble, dim3(G.nn, cg), dim3(64), 0, st, G.dev, s->dev, X, d_w,
                           w_stride, d_status);
        if ((rc = launch_check("pf_se_estimate: assemble"))) return rc;
        // G is symmetric: the lower blocks alone take the updates
        factor_launch(G, B, X.vals, X.vs, kSeGroup, nullptr, st, true);
        if ((rc = launch_check("pf_se_estimate: factor"))) return rc;
        if ((rc = pf_solve(&s->gain, B, X.vals, X.vs, kSeGroup, X.rhs, X.rs, 0, stream)))
            return rc;
        hipLaunchKernelGGL(k_se_update, dim3(B), dim3(256), 0, st, G.dev, s->dev, X, d_Vm, d_Va,
                           v_stride, tol, it, max_iter, d_iters, d_norm, d_status);
        if ((rc = launch_check("pf_se_estimate: update"))) return rc;
        rc = hip_check(hipMemcpyAsync(host.data(), d_status, sizeof(int32_t) * B,
                                      hipMemcpyDeviceToHost, st),
                       "pf_se_estimate: status copy");
        if (rc) return rc;
        if ((rc = hip_check(hipStreamSynchronize(st), "pf_se_estimate: sync"))) return rc;
        bool all = true;
        for (int c = 0; c < B; ++c) all = all && host[c] >= 0;
        if (all) break;
    }
    return PF_OK;
}

void pf_se_destroy(pf_se s) { delete s; }


}  // extern "C"
