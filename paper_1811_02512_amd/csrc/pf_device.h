// libpf device-side building blocks shared by the kernel files (gfx950):
// views of the interleaved workspaces, 2x2 block helpers, level loops,
// the factor / solve node routines, the LDS tail and the mismatch pass.
// Included by every .hip file of the library; everything here has
// internal linkage (one copy per translation unit).
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
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "pf.h"
#include "pf_internal.h"
#include "pf_kernels.h"

// The library's internal headers work in namespace pf.
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
// Value of the workgroup's zero-pivot marker while no pivot has failed; a
// failing pivot lowers it to its node's level-ordered index, so that the
// marker ends at the first failure in level order, then ascending position
// (the order of a sequential factorisation over the partition).
constexpr int kNoPivot = 0x7fffffff;

__device__ __forceinline__ void mark_pivot(int* s_bad, int x) { atomicMin(s_bad, x); }

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
    // the right-hand side of the Newton step sits in the bus record beside P, Q
    static constexpr bool kRhsInRecord = true;
    struct DiagIn {
        double2 y;
        Blk r;  // e, f, |V|, theta of the node's bus
        double2 s;  // P, Q
        double2 f;  // F_P, F_Q (the rhs)
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
        const Blk pqf = w.blk(rec + 4);  // P, Q, F_P, F_Q
        return {y2[yd], r, {pqf.a, pqf.b}, {pqf.c, pqf.d}, type(bus)};
    }
    __device__ __forceinline__ double2 rhs_at(int bus) const
    {
        return w.v2(bus_off + 8 * (int64_t)bus + 6);
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
    static constexpr bool kRhsInRecord = false;
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

// Level-ordered node record, the part the sweeps use ({j, bus, r0, r1},
// {s0, s1, ydiag, 0}); the admittance-row range is read by the mismatch only.
struct NodeRec {
    int4 a, b;
};

__device__ __forceinline__ NodeRec load_rec(const DevSym& S, int x)
{
    return {S.node_info[3 * x], S.node_info[3 * x + 1]};
}

// How one case's work is split over the workgroups of a launch.
// OneGroup: the whole case in one workgroup, levels separated by workgroup
// barriers.
struct OneGroup {
    static constexpr bool kSpread = false;
    static constexpr bool kSub = false;
    __device__ __forceinline__ int rank() const { return 0; }
    __device__ __forceinline__ int size() const { return 1; }
    __device__ __forceinline__ void sync() const { __syncthreads(); }
};

// Spread: the case's wide phases (loops over buses, the levels below the LDS
// tail) over the workgroups of a cooperative launch that own the case (all
// of them, or a group in a batch of grids), which meet at grid barriers;
// the tail stays on the group's first workgroup while the others wait.  The
// barrier words live in three 128-byte lines of the case's workspace,
// zeroed (the pivot marker set to kNoPivot) before the launch:
//   line 0: arrivals (count of workgroups that reached a barrier, over all
//           barriers so far); line 1: release (number of the last barrier
//           every workgroup has reached); line 2: abort flag, zero-pivot
//           marker, then per parity of the iteration count a NaN flag and
//           the bits of the mismatch maximum (a non-negative double, whose
//           bit patterns order as unsigned integers do).
// A workgroup makes its writes visible before it arrives (an agent-scope
// release fence: its XCD's L2 written back) and discards stale cached lines
// after it is released (an agent-scope acquire fence), so what any workgroup
// wrote before a barrier is what every workgroup reads after it: each
// arrival is counted only after its writes have reached memory, the release
// word is stored only after every arrival has been counted, and a workgroup
// reads only after it has seen the release word and invalidated its caches.
// A wait that lasts longer than wait_ticks of the constant 100 MHz clock
// (one second unless a caller lowers it) sets the abort flag; from then on
// no barrier waits, so every workgroup runs to its end and the case reports
// the failure.
constexpr int kSpreadWords = 96;  // 32-bit words of the three lines

struct Spread {
    static constexpr bool kSpread = true;
    static constexpr bool kSub = false;  // every level below the tail shared
    unsigned* arrive;
    unsigned* release;
    int* flags;        // abort, pivot marker, NaN flag [2]
    uint64_t* maxbits; // [2]
    unsigned* count;   // LDS: barriers this workgroup has passed
    // levels [back_lo, tail level) of the backward substitution run on
    // workgroup 0 right after the tail's (narrow levels: workgroup barriers
    // are cheaper there than grid barriers)
    int back_lo;
    unsigned long long wait_ticks;
    int rk, sz;  // this workgroup's rank in the case's group, the group's size
    __device__ __forceinline__ int rank() const { return rk; }
    __device__ __forceinline__ int size() const { return sz; }
    __device__ __forceinline__ int* marker() const { return flags + 1; }
    __device__ __forceinline__ bool aborted() const
    {
        return __hip_atomic_load(flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    }
    __device__ __forceinline__ void sync() const
    {
        __syncthreads();
        if (threadIdx.x == 0) {
            const unsigned k = ++*count;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            const unsigned before =
                __hip_atomic_fetch_add(arrive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (!aborted()) {
                if (before == k * (unsigned)sz - 1) {
                    __hip_atomic_store(release, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                } else {
                    const unsigned long long t0 = wall_clock64();
                    while (__hip_atomic_load(release, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT) < k) {
                        if (aborted()) break;
                        if (wall_clock64() - t0 > wait_ticks) {
                            __hip_atomic_store(flags, 1, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
    }
};

// As Spread, with the levels below the subtree cut (DevSym::sub_cut) run by
// each workgroup on whole subtrees of its own, workgroup barriers between
// them: used by the groups of a batch of grids, where grid barriers contend
// with the other groups for the XCDs they share.  (One case alone keeps
// Spread: there the subtree levels measured slower than shared ones.)
struct SpreadSub : Spread {
    static constexpr bool kSub = true;
};

// Runs fn(x, rec, lane, g) for the nodes of levels [l0, l1), up or down,
// with a barrier of the split after every level: x indexes the level-ordered
// node records, rec is x's record, and each node gets g lanes (the level's
// mapping); the groups of g lanes of all the split's workgroups take the
// level's nodes in turn, group k of every workgroup before group k + 1 of
// any, so that a narrow level still reaches every workgroup.  The record of
// the group's next node in the level is fetched before fn runs so that its
// latency overlaps the current node's work.
template <class P, class F>
__device__ __forceinline__ void for_nodes(const P& par, const DevSym& S, int l0, int l1, bool up,
                                          F&& fn)
{
    for (int li = l0; li < l1; ++li) {
        const int l = up ? li : l1 - 1 - (li - l0);
        const int g = S.level_g[l];
        const int beg = S.level_ptr[l];
        const int cnt = S.level_ptr[l + 1] - beg;
        const int gpb = blockDim.x / g;
        const int step = gpb * par.size();
        const int lane = threadIdx.x & (g - 1);
        int idx = (int)(threadIdx.x / g) * par.size() + par.rank();
        NodeRec cur = idx < cnt ? load_rec(S, beg + idx) : NodeRec{};
        while (idx < cnt) {
            const int nxt = idx + step;
            const NodeRec pre = nxt < cnt ? load_rec(S, beg + nxt) : NodeRec{};
            fn(beg + idx, cur, lane, g);
            cur = pre;
            idx = nxt;
        }
        par.sync();
    }
}

template <class F>
__device__ __forceinline__ void for_nodes(const DevSym& S, int l0, int l1, bool up, F&& fn)
{
    for_nodes(OneGroup{}, S, l0, l1, up, static_cast<F&&>(fn));
}

// As for_nodes over levels [l0, l1) below the subtree cut, for the nodes of
// this workgroup's subtrees only (roots [k0, k1)), with a workgroup barrier
// after every level: a node's descendants belong to its own subtree, so no
// other workgroup's results are needed until the cut.
template <class F>
__device__ __forceinline__ void for_sub_levels(const DevSym& S, int k0, int k1, int l0, int l1,
                                               bool up, F&& fn)
{
    const int R1 = S.sub_roots + 1;
    for (int li = l0; li < l1; ++li) {
        const int l = up ? li : l1 - 1 - (li - l0);
        const int g = S.level_g[l];
        const int b = S.level_ptr[l];
        const int e1 = b + S.sub_ptr[l * R1 + k1];
        const int gpb = blockDim.x / g;
        const int lane = threadIdx.x & (g - 1);
        int e = b + S.sub_ptr[l * R1 + k0] + (int)threadIdx.x / g;
        int x = e < e1 ? S.sub_idx[e] : 0;
        NodeRec cur = e < e1 ? load_rec(S, x) : NodeRec{};
        while (e < e1) {
            const int en = e + gpb;
            const int xn = en < e1 ? S.sub_idx[en] : 0;
            const NodeRec pre = en < e1 ? load_rec(S, xn) : NodeRec{};
            fn(x, cur, lane, g);
            cur = pre;
            x = xn;
            e = en;
        }
        __syncthreads();
    }
}

// The subtrees [k0, k1) of workgroup `rank` of `size`: the roots whose work
// starts in its share [rank, rank + 1) / size of the total (every workgroup
// of the group calls this; k0 = k1 = 0 without subtrees).
template <class P>
__device__ __forceinline__ void sub_share(const DevSym& S, const P& par, int& k0, int& k1)
{
    __shared__ int s_k[2];
    k0 = k1 = 0;
    if (S.sub_cut <= 0) return;
    if (threadIdx.x < 2) s_k[threadIdx.x] = 0;
    __syncthreads();
    const int R = S.sub_roots;
    const int64_t tot = S.sub_cum[R];
    const int64_t a = tot * par.rank() / par.size();
    const int64_t b = tot * (par.rank() + 1) / par.size();
    int c0 = 0, c1 = 0;
    for (int k = threadIdx.x; k < R; k += blockDim.x) {
        const int64_t v = S.sub_cum[k];
        c0 += v < a;
        c1 += v < b;
    }
    if (c0) atomicAdd(&s_k[0], c0);
    if (c1) atomicAdd(&s_k[1], c1);
    __syncthreads();
    k0 = s_k[0];
    k1 = s_k[1];
    __syncthreads();
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
// step's blocks so that index and value loads overlap.  Pairs past the end
// of a list are not loaded (a load no lane of the wavefront needs is
// skipped) and contribute nothing.
__device__ __forceinline__ int2 upd_at(const int2* __restrict__ upd, int u, int u1)
{
    int2 p = make_int2(0, 0);
    if (u < u1) p = upd[u];
    return p;
}

// The four blocks pair p reads: W_a = W(p.x), U_a = U(p.x), W_b, U_b of p.y.
struct PairBlk {
    Blk Wa, Ua, Wb, Ub;
};
__device__ __forceinline__ PairBlk pair_blocks(const View& w, int64_t lu, int2 p, bool has)
{
    PairBlk b{bzero(), bzero(), bzero(), bzero()};
    if (has) {
        b.Wa = w.blk(lu + 8 * (int64_t)p.x);
        b.Ua = w.blk(lu + 8 * (int64_t)p.x + 4);
        b.Wb = w.blk(lu + 8 * (int64_t)p.y);
        b.Ub = w.blk(lu + 8 * (int64_t)p.y + 4);
    }
    return b;
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
        const PairBlk a = pair_blocks(w, lu, p, true);
        const PairBlk c = pair_blocks(w, lu, q, has_q);
        bmsub(Wk, a.Wa, a.Ub);
        bmsub(Vk, a.Wb, a.Ua);
        if (has_q) {
            bmsub(Wk, c.Wa, c.Ub);
            bmsub(Vk, c.Wb, c.Ua);
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
            Blk Wa = bzero(), Ub = bzero(), Wc = bzero(), Ud = bzero();
            if (hp) {
                Wa = w.blk(lu + 8 * (int64_t)p.x);
                Ub = w.blk(lu + 8 * (int64_t)p.y + 4);
            }
            if (hq) {
                Wc = w.blk(lu + 8 * (int64_t)q.x);
                Ud = w.blk(lu + 8 * (int64_t)q.y + 4);
            }
            if (hp) bmsub(Wk, Wa, Ub);
            if (hq) bmsub(Wk2, Wc, Ud);
        } else {
            const PairBlk x = pair_blocks(w, lu, p, hp);
            const PairBlk y = pair_blocks(w, lu, q, hq);
            if (hp) {
                bmsub(Wk, x.Wa, x.Ub);
                bmsub(Vk, x.Wb, x.Ua);
            }
            if (hq) {
                bmsub(Wk2, y.Wa, y.Ub);
                bmsub(Vk2, y.Wb, y.Ua);
            }
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

// Updates of one tail destination from its packed local pair list (np
// pairs starting at load l, the first two loads q0, q1 already requested):
// eight pairs per step, the next two loads in flight; updates in list order.
__device__ __forceinline__ void apply_packed_lds(const uint4* __restrict__ pk, int l, int np,
                                                 uint4 q0, uint4 q1, const double* sLU, Blk& Wk,
                                                 Blk& Vk)
{
    for (int k = 0; k < np; k += 8) {
        const int i = l + (k >> 2);
        uint4 n0 = make_uint4(0, 0, 0, 0), n1 = n0;
        if (k + 8 < np) n0 = pk[i + 2];
        if (k + 12 < np) n1 = pk[i + 3];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            if (k + c < np) {
                const uint32_t v = pk_word(c < 4 ? q0 : q1, c & 3);
                const int a = v & 0xffff, b = v >> 16;
                bmsub(Wk, bload(sLU + 8 * a), bload(sLU + 8 * b + 4));
                bmsub(Vk, bload(sLU + 8 * b), bload(sLU + 8 * a + 4));
            }
        }
        q0 = n0;
        q1 = n1;
    }
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

// Group sums of a block and, with rhs, of a 2-vector, all six interleaved.
__device__ __forceinline__ void gsum_blk(Blk& v, double& z0, double& z1, bool rhs, int g)
{
    if (rhs) {
        double t[6] = {v.a, v.b, v.c, v.d, z0, z1};
        gsum_n(t, g);
        v = {t[0], t[1], t[2], t[3]};
        z0 = t[4];
        z1 = t[5];
    } else {
        double t[4] = {v.a, v.b, v.c, v.d};
        gsum_n(t, g);
        v = {t[0], t[1], t[2], t[3]};
    }
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
// update chains in flight together.  Absent list entries, slots and update
// pairs are not loaded (a load no lane of the wavefront needs is skipped)
// and add nothing.
// SYM: a symmetric matrix (eq. 2 blockwise): only the lower blocks take
// updates and U_jk = D_j^-1 W_kj^T.
// x: the node's level-ordered index (for the zero-pivot marker s_bad).
template <class SRC, bool FWD, bool STORE_D, bool SYM = false>
__device__ __forceinline__ void factor_node(const DevSym& S, const SRC& src, int x,
                                            const NodeRec& rec, int lane, int g, const View& w,
                                            int64_t lu, const View& wr, int64_t rhs, int* s_bad)
{
    const int4 n0 = rec.a;
    const int4 n1 = rec.b;
    const int j = n0.x, bus = n0.y;
    const int r1 = n0.w, s1 = n1.y;
    const typename SRC::DiagIn din = src.diag_in(j, bus, n1.z);
    double2 bj = make_double2(0.0, 0.0);
    if constexpr (FWD) {
        if constexpr (SRC::kRhsInRecord) bj = din.f;
        else bj = wr.v2(rhs + 2 * (int64_t)j);
    }
    // Absent list entries are not loaded at all (each guarded load is skipped
    // when no lane of the wavefront needs it: the sweeps are bound by the
    // number of vector-memory instructions, not by bytes).
    int s = n1.x + lane;
    const int4 z4 = make_int4(0, 0, 0, 0);
    int4 sa = z4, sb = z4, sa2 = z4, sb2 = z4;
    if (s < s1) {
        sa = S.slot_info[2 * s];
        sb = S.slot_info[2 * s + 1];
    }
    if (s + g < s1) {
        sa2 = S.slot_info[2 * (s + g)];
        sb2 = S.slot_info[2 * (s + g) + 1];
    }
    int2 e[4];
    int r = n0.z + lane;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        e[k] = make_int2(0, 0);
        if (r + k * g < r1) e[k] = S.rl[r + k * g];
    }
    Blk ds = bzero();
    double z0 = 0.0, z1 = 0.0;
    for (; r < r1; r += 4 * g) {
        Blk wv[4], uv[4];
        double2 yi[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            wv[k] = bzero();
            uv[k] = bzero();
            yi[k] = make_double2(0.0, 0.0);
            if (r + k * g < r1) {
                wv[k] = w.blk(lu + 8 * (int64_t)e[k].y);
                uv[k] = w.blk(lu + 8 * (int64_t)e[k].y + 4);
                if (FWD) yi[k] = wr.v2(rhs + 2 * (int64_t)e[k].x);
            }
        }
        const int rn = r + 4 * g;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (rn + k * g < r1) e[k] = S.rl[rn + k * g];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (r + k * g < r1) {
                bmadd(ds, wv[k], uv[k]);
                if (FWD) mvadd(z0, z1, wv[k], yi[k].x, yi[k].y);
            }
        }
    }
    if (g > 1) {
        gsum_blk(ds, z0, z1, FWD, g);
    }
    const Blk Ajj = src.diag_of(din);
    bool ok;
    const Blk Di = binv({Ajj.a - ds.a, Ajj.b - ds.b, Ajj.c - ds.c, Ajj.d - ds.d}, ok);
    for (; s < s1; s += 2 * g) {
        const int s2 = s + g;
        const bool two = s2 < s1;
        const typename SRC::OffIn o1 = src.off_in(s, sa.y, sa.z, sa.w);
        typename SRC::OffIn o2{};
        if (two) o2 = src.off_in(s2, sa2.y, sa2.z, sa2.w);
        const int u0 = sb.x, u1 = sb.y, v0 = two ? sb2.x : 0, v1 = two ? sb2.y : 0;
        int2 p = make_int2(0, 0), q = make_int2(0, 0);
        if (u0 < u1) p = S.upd[u0];
        if (v0 < v1) q = S.upd[v0];
        const int sn = s + 2 * g;
        if (sn < s1) {
            sa = S.slot_info[2 * sn];
            sb = S.slot_info[2 * sn + 1];
        }
        if (sn + g < s1) {
            sa2 = S.slot_info[2 * (sn + g)];
            sb2 = S.slot_info[2 * (sn + g) + 1];
        }
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
        if (!ok) mark_pivot(s_bad, x);
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
// With a Spread split, every workgroup of the launch takes a share of phase
// A and leaves its results in the tail's own places in global memory (the
// D blocks, rhs entries and slot records of the tail nodes, which nothing
// else reads until the tail writes them); after a grid barrier workgroup 0
// loads them into LDS and runs the rest, and the other workgroups return.
template <class SRC, bool FWD, bool WRITE, class P = OneGroup>
__device__ __forceinline__ void tail_factor(const DevSym& S, const SRC& src, const View& w,
                                            int64_t lu, const View& wr, int64_t rhs, int* s_bad,
                                            const P& par = P{})
{
    const int K = S.tail_nodes, TS = S.tail_slots, KC = S.tail_clique;
    const int nT = S.nlev - S.tail_level;
    double* sLU = pf_smem;             // TS x 8: W, then V -> U
    double* sD = pf_smem + 8 * TS;     // K x 4: accumulated pivot, then D^-1
    double* sy = sD + 4 * K;           // K x 2: accumulated rhs, then y
    const int a0 = P::kSpread ? par.rank() * (int)blockDim.x + (int)threadIdx.x : threadIdx.x;
    const int as = P::kSpread ? par.size() * (int)blockDim.x : blockDim.x;
    for (int it = a0; it < K + TS; it += as) {
        if (it < K) {
            const int4 t0 = S.t_node[3 * it];
            const int4 t1 = S.t_node[3 * it + 1];
            Blk acc = src.diag(t0.x, t0.y, t0.z);
            double z0 = 0.0, z1 = 0.0;
            if constexpr (FWD) {
                double2 b;
                if constexpr (SRC::kRhsInRecord) b = src.rhs_at(t0.y);
                else b = wr.v2(rhs + 2 * (int64_t)t0.x);
                z0 = b.x;
                z1 = b.y;
            }
            // lower neighbours outside the tail: four per step, their blocks
            // and y requested together, the next four indices in flight
            // (entries past the list's end are not loaded)
            if (t1.y < t1.z) {
                int2 e[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) e[k] = upd_at(S.t_rl, t1.y + k, t1.z);
                for (int r = t1.y; r < t1.z; r += 4) {
                    int2 nx[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) nx[k] = upd_at(S.t_rl, r + 4 + k, t1.z);
                    Blk wv[4], uv[4];
                    double2 yi[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        wv[k] = bzero();
                        uv[k] = bzero();
                        yi[k] = make_double2(0.0, 0.0);
                        if (r + k < t1.z) {
                            wv[k] = w.blk(lu + 8 * (int64_t)e[k].y);
                            uv[k] = w.blk(lu + 8 * (int64_t)e[k].y + 4);
                            if (FWD) yi[k] = wr.v2(rhs + 2 * (int64_t)e[k].x);
                        }
                    }
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        if (r + k < t1.z) {
                            bmsub(acc, wv[k], uv[k]);
                            if (FWD) {
                                z0 = fma(-wv[k].a, yi[k].x, fma(-wv[k].b, yi[k].y, z0));
                                z1 = fma(-wv[k].c, yi[k].x, fma(-wv[k].d, yi[k].y, z1));
                            }
                        }
                    }
#pragma unroll
                    for (int k = 0; k < 4; ++k) e[k] = nx[k];
                }
            }
            if constexpr (P::kSpread) {
                w.put(4 * (int64_t)t0.x, acc);
                if (FWD) wr.put2(rhs + 2 * (int64_t)t0.x, make_double2(z0, z1));
            } else {
                bstore(sD + 4 * it, acc);
                sy[2 * it] = z0;
                sy[2 * it + 1] = z1;
            }
        } else {
            const int t = it - K;
            const int4 a = S.t_slot[3 * t];
            const int4 b = S.t_slot[3 * t + 1];
            const int4 c = S.t_slot[3 * t + 2];
            Blk Wk, Vk;
            src.off(a.x, c.x, a.z, a.w, b.x, Wk, Vk);
            apply_updates(S.t_upd, b.y, b.z, w, lu, Wk, Vk);
            if constexpr (P::kSpread) {
                w.put(lu + 8 * (int64_t)a.x, Wk);
                w.put(lu + 8 * (int64_t)a.x + 4, Vk);
            } else {
                bstore(sLU + 8 * t, Wk);
                bstore(sLU + 8 * t + 4, Vk);
            }
        }
    }
    if constexpr (P::kSpread) {
        par.sync();
        if (par.rank() != 0) return;
        for (int it = threadIdx.x; it < K + TS; it += blockDim.x) {
            if (it < K) {
                const int j = S.t_node[3 * it].x;
                bstore(sD + 4 * it, w.blk(4 * (int64_t)j));
                const double2 z = FWD ? wr.v2(rhs + 2 * (int64_t)j) : make_double2(0.0, 0.0);
                sy[2 * it] = z.x;
                sy[2 * it + 1] = z.y;
            } else {
                const int t = it - K;
                const int64_t sg = lu + 8 * (int64_t)S.t_slot[3 * t].x;
                bstore(sLU + 8 * t, w.blk(sg));
                bstore(sLU + 8 * t + 4, w.blk(sg + 4));
            }
        }
    }
    __syncthreads();
    // Each level's node records arrive before its barrier; a lane's first
    // slot record and that slot's first packed pair loads are requested
    // before the lower-neighbour sums, so the slot loop starts on indices
    // already in registers.
    for_tail_pf(S, 0, nT - KC, true, [&](int jl, const int4& t0, const int4& t1, const int4&,
                                         int lane, int g) {
        const int4 z4 = make_int4(0, 0, 0, 0);
        const uint4 zq = make_uint4(0, 0, 0, 0);
        int t = t0.w + lane;
        int4 sb = z4, sc = z4;
        if (t < t1.x) {
            sb = S.t_slot[3 * t + 1];
            sc = S.t_slot[3 * t + 2];
        }
        int r = t1.z + lane;
        int2 e = make_int2(0, 0);
        if (r < t1.w) e = S.t_rl[r];
        int np = sb.w - sb.z;
        uint4 q0 = zq, q1 = zq;
        if (np > 0) q0 = S.t_pk[sc.w];
        if (np > 4) q1 = S.t_pk[sc.w + 1];
        Blk ds = bzero();
        double z0 = 0.0, z1 = 0.0;
        for (; r < t1.w; r += g) {
            const int2 en = upd_at(S.t_rl, r + g, t1.w);
            const Blk wv = bload(sLU + 8 * e.y);
            bmadd(ds, wv, bload(sLU + 8 * e.y + 4));
            if (FWD) mvadd(z0, z1, wv, sy[2 * e.x], sy[2 * e.x + 1]);
            e = en;
        }
        if (g > 1) {
            gsum_blk(ds, z0, z1, FWD, g);
        }
        const Blk A = bload(sD + 4 * jl);
        bool ok;
        const Blk Di = binv({A.a - ds.a, A.b - ds.b, A.c - ds.c, A.d - ds.d}, ok);
        for (; t < t1.x; t += g) {
            const int tn = t + g;
            int4 sbn = z4, scn = z4;
            if (tn < t1.x) {
                sbn = S.t_slot[3 * tn + 1];
                scn = S.t_slot[3 * tn + 2];
            }
            Blk Wk = bload(sLU + 8 * t), Vk = bload(sLU + 8 * t + 4);
            apply_packed_lds(S.t_pk, sc.w, np, q0, q1, sLU, Wk, Vk);
            bstore(sLU + 8 * t, Wk);
            bstore(sLU + 8 * t + 4, bmul(Di, Vk));
            sc = scn;
            np = sbn.w - sbn.z;
            q0 = zq;
            q1 = zq;
            if (np > 0) q0 = S.t_pk[sc.w];
            if (np > 4) q1 = S.t_pk[sc.w + 1];
        }
        if (lane == 0) {
            if (!ok) mark_pivot(s_bad, S.level_ptr[S.tail_level] + jl);
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
                if (!ok && threadIdx.x == 0) mark_pivot(s_bad, S.level_ptr[S.tail_level] + ja);
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
__device__ __forceinline__ void tail_backward(const DevSym& S, const View& w, int64_t rhs,
                                              int64_t bus_off, PvMask type, double2* xs)
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
            gsum2(a0, a1, g);
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
    // absent entries are not loaded (skipped when no lane needs them)
    int s = n1.x + lane;
    int kk[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        kk[k] = 0;
        if (s + k * g < s1) kk[k] = S.Li[s + k * g];
    }
    double a0 = 0.0, a1 = 0.0;
    for (; s < s1; s += 4 * g) {
        Blk u[4];
        double2 xk[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            u[k] = bzero();
            xk[k] = make_double2(0.0, 0.0);
            if (s + k * g < s1) {
                u[k] = w.blk(lu + 8 * (int64_t)(s + k * g) + 4);
                xk[k] = xs ? xs[kk[k]] : wb.v2(rhs + 2 * (int64_t)kk[k]);
            }
        }
        const int sn = s + 4 * g;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (sn + k * g < s1) kk[k] = S.Li[sn + k * g];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (s + k * g < s1) mvadd(a0, a1, u[k], xk[k].x, xk[k].y);
    }
    if (g > 1) {
        gsum2(a0, a1, g);
    }
    if (lane == 0) {
        const double x0 = y.x - a0, x1 = y.y - a1;
        if (xs) xs[n0.x] = make_double2(x0, x1);
        else wb.put2(rhs + 2 * (int64_t)n0.x, make_double2(x0, x1));
        if (UPDATE) apply_step_to(wb, brec, br, pv, x0, x1);
    }
}

// Max over the workgroup with a NaN flag; every thread gets the result.
__device__ __forceinline__ double block_max(double v, int nan, int& any_nan)
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
    int32_t* pivot;  // position of the first zero pivot, -1 if none (may be null)
};

// Arguments of the fused adjoint kernel (pf_adjoint).
struct AdjArgs {
    double* ws;  // pf_newton's workspace: factors of J at the solution
    int64_t ws_stride;
    int C;  // interleave of the workspace
    int B;
    const double* gVm;  // dL/d|V| [B][n] or null
    const double* gVa;  // dL/dtheta [B][n] or null
    int64_t gv_stride;
    const int8_t* type;
    int64_t type_stride;
    const int32_t* status;  // pf_newton's per-case status or null
    double* lam;            // out: adjoint vector [B][nn][2]
    int64_t lam_stride;
    double* gP;
    double* gQ;
    int64_t g_stride;
    // branch gradients in the same launch (gx null: none)
    const int32_t* from;
    const int32_t* to;
    const double* Vm;
    const double* Va;
    int64_t v_stride;
    const double* r;
    const double* x;
    int64_t branch_stride;
    double* gx;   // gx_mode 0: dL/dx [B][m]; 1: null here, per-case parts to the workspace
    int gx_mode;  // 0 per case, 1 summed over the cases (by k_adj_gx_sum)
};

struct CaseDesc {
    DevSym sym;
    int64_t bus_off, br_off, y_off, ws_off;
    // a batch of grids spread over more workgroups than cases: this case's
    // workgroup count, its grid-barrier words (doubles after ws_off) and the
    // first backward level left to its first workgroup
    int64_t sync_off;
    int32_t spread, back_lo;
};

// Mismatch pass of one case: F = calculated - scheduled (F_Q = 0 at PV buses)
// and P + jQ.  Without SCALE (Newton) P, Q, F_P, F_Q go into the second half
// of the bus record in one store; with SCALE (the fast decoupled right-hand
// sides) P, Q into the record and F / |V| into the rhs in position order.  The thread's max
// |F| and NaN flag accumulate into mx and nan.  Buses are taken in bus
// order, NB per thread per step (blockDim apart), so that the admittance
// rows, row pointers, positions and scheduled injections of a wavefront are
// adjacent in memory; all loads of a step's buses are issued before any of
// them is summed.  The buses are first, first + stride, ... (the thread's
// index and count over the workgroups that share the case).
template <bool SCALE, class EF, int NB = 2>
__device__ __forceinline__ void mismatch_pass(const DevSym& S, const double* yv, const EF& ef,
                                              const View& wb, const Off& o, const PvMask& pvm,
                                              const double* Psp, const double* Qsp, double& mx,
                                              int& nan, int first, int stride)
{
    const int bd = stride;
    for (int i0 = first; i0 < S.n; i0 += NB * bd) {
        int ib[NB], pc[NB], q0[NB], q1[NB];
        bool has[NB], pv[NB];
        double sp[NB], sq[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            has[k] = i0 + k * bd < S.n;
            ib[k] = has[k] ? i0 + k * bd : i0;
            pc[k] = S.pos[ib[k]];
            q0[k] = S.yptr[ib[k]];
            q1[k] = S.yptr[ib[k] + 1];
            sp[k] = Psp[ib[k]];
            sq[k] = Qsp[ib[k]];
        }
        Blk v[NB];  // e, f, |V| (|V| only with SCALE)
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            if (SCALE) {
                v[k] = wb.blk(o.BUS + 8 * (int64_t)ib[k]);
            } else {
                ef.get(ib[k], v[k].a, v[k].b);
                v[k].c = 1.0;
            }
            pv[k] = pvm(ib[k]);
        }
        int kk[NB][4];
        RowHead h[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) row_head_idx<EF>(S, yv, q0[k], q1[k], kk[k], h[k]);
#pragma unroll
        for (int k = 0; k < NB; ++k) row_head_v(ef, kk[k], h[k]);
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            double p, q;
            row_finish(S, yv, ef, q0[k], q1[k], h[k], v[k].a, v[k].b, p, q);
            if (has[k] && pc[k] >= 0) {  // the slack is not a position
                const int64_t rc = o.BUS + 8 * (int64_t)ib[k];
                const double fp = p - sp[k], fq = pv[k] ? 0.0 : q - sq[k];
                if (SCALE) {
                    wb.put2(rc + 4, make_double2(p, q));
                    wb.put2(o.RHS + 2 * (int64_t)pc[k], make_double2(fp / v[k].c, fq / v[k].c));
                } else {  // P, Q and the Newton rhs F in one store of the bus record
                    wb.put(rc + 4, {p, q, fp, fq});
                }
                nan |= (fp != fp) | (fq != fq);
                mx = fmax(mx, fmax(fabs(fp), fabs(fq)));
            }
        }
    }
}

template <bool SCALE, class EF, int NB = 2>
__device__ __forceinline__ void mismatch_pass(const DevSym& S, const double* yv, const EF& ef,
                                              const View& wb, const Off& o, const PvMask& pvm,
                                              const double* Psp, const double* Qsp, double& mx,
                                              int& nan)
{
    mismatch_pass<SCALE, EF, NB>(S, yv, ef, wb, o, pvm, Psp, Qsp, mx, nan, (int)threadIdx.x,
                                 (int)blockDim.x);
}

}  // namespace
