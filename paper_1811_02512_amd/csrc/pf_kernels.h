// Device building blocks of the level-scheduled Newton-Raphson power flow.
// gfx950, fp64, 64-wide wavefronts.  No atomics on values: every output word
// has one writer, so results are bitwise reproducible.
#pragma once

#include <hip/hip_runtime.h>

#include "pf_internal.h"

namespace pf {

enum : int { ST_OK = 0, ST_ZERO_PIVOT = 5, ST_NOT_CONVERGED = 6, ST_NONFINITE = 7 };
enum : int8_t { T_PQ = 1, T_PV = 2, T_SLACK = 3 };

// 2x2 block, row-major.
struct Blk {
    double a, b, c, d;
};

__device__ __forceinline__ Blk bzero() { return {0.0, 0.0, 0.0, 0.0}; }

__device__ __forceinline__ Blk bload(const double* __restrict__ p)
{
    const double2* q = reinterpret_cast<const double2*>(p);
    double2 x = q[0], y = q[1];
    return {x.x, x.y, y.x, y.y};
}

__device__ __forceinline__ void bstore(double* __restrict__ p, const Blk& v)
{
    double2* q = reinterpret_cast<double2*>(p);
    q[0] = make_double2(v.a, v.b);
    q[1] = make_double2(v.c, v.d);
}

// acc += x * y
__device__ __forceinline__ void bmadd(Blk& acc, const Blk& x, const Blk& y)
{
    acc.a = fma(x.a, y.a, fma(x.b, y.c, acc.a));
    acc.b = fma(x.a, y.b, fma(x.b, y.d, acc.b));
    acc.c = fma(x.c, y.a, fma(x.d, y.c, acc.c));
    acc.d = fma(x.c, y.b, fma(x.d, y.d, acc.d));
}

// acc -= x * y
__device__ __forceinline__ void bmsub(Blk& acc, const Blk& x, const Blk& y)
{
    acc.a = fma(-x.a, y.a, fma(-x.b, y.c, acc.a));
    acc.b = fma(-x.a, y.b, fma(-x.b, y.d, acc.b));
    acc.c = fma(-x.c, y.a, fma(-x.d, y.c, acc.c));
    acc.d = fma(-x.c, y.b, fma(-x.d, y.d, acc.d));
}

__device__ __forceinline__ Blk bmul(const Blk& x, const Blk& y)
{
    Blk r = bzero();
    bmadd(r, x, y);
    return r;
}

__device__ __forceinline__ Blk btrans(const Blk& x) { return {x.a, x.c, x.b, x.d}; }

// y += A x ; y += A^T x
__device__ __forceinline__ void mvadd(double& y0, double& y1, const Blk& A, double x0, double x1)
{
    y0 = fma(A.a, x0, fma(A.b, x1, y0));
    y1 = fma(A.c, x0, fma(A.d, x1, y1));
}
__device__ __forceinline__ void mtvadd(double& y0, double& y1, const Blk& A, double x0, double x1)
{
    y0 = fma(A.a, x0, fma(A.c, x1, y0));
    y1 = fma(A.b, x0, fma(A.d, x1, y1));
}

// Inverse of a 2x2 block; ok = false when the determinant is zero or not finite.
__device__ __forceinline__ Blk binv(const Blk& x, bool& ok)
{
    double det = x.a * x.d - x.b * x.c;
    ok = (det != 0.0) && isfinite(det);
    double r = 1.0 / det;
    return {x.d * r, -x.b * r, -x.c * r, x.a * r};
}

// The value of the lane that DPP control CTRL selects (all rows and banks;
// the selected lane always lies in the caller's lane group).
template <int CTRL>
__device__ __forceinline__ double dpp_peer(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// The value of lane (i xor 16) within each half-wavefront (swizzle, bit mode:
// and-mask 31, or-mask 0, xor-mask 16).
__device__ __forceinline__ double swz_xor16(double v)
{
    const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), 0x401F);
    const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), 0x401F);
    return __hiloint2double(hi, lo);
}

// Sums of N values over the g lanes of a lane group (g a power of two <= 64,
// groups aligned inside the wavefront), the N reductions interleaved.
// Butterfly with partners inside a row of 16 lanes taken by DPP moves (no
// LDS round trip): lane xor 1 and xor 2 of a quad, then the mirrored lane
// within 8 and within 16, which after the earlier steps holds the other
// half's partial sum; across rows lane xor 16 (swizzle) and xor 32
// (permute).  Each step adds the same two operands on both lanes of a pair,
// so every lane of a group ends with the same bits.
template <int N>
__device__ __forceinline__ void gsum_n(double (&v)[N], int g)
{
    if (g >= 2) {
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] += dpp_peer<0xB1>(v[k]);  // quad_perm 1,0,3,2
    }
    if (g >= 4) {
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] += dpp_peer<0x4E>(v[k]);  // quad_perm 2,3,0,1
    }
    if (g >= 8) {
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] += dpp_peer<0x141>(v[k]);  // row_half_mirror
    }
    if (g >= 16) {
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] += dpp_peer<0x140>(v[k]);  // row_mirror
    }
    if (g >= 32) {
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] += swz_xor16(v[k]);
    }
    if (g >= 64) {
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] += __shfl_xor(v[k], 32, 64);
    }
}

__device__ __forceinline__ double gsum(double v, int g)
{
    double t[1] = {v};
    gsum_n(t, g);
    return t[0];
}

// Two sums at once (a 2-vector spread over the group).
__device__ __forceinline__ void gsum2(double& a, double& b, int g)
{
    double t[2] = {a, b};
    gsum_n(t, g);
    a = t[0];
    b = t[1];
}

// Off-diagonal Jacobian block (i, k) = d(P_i, Q_i)/d(theta_k, |V_k|) from
// Y_ik = G + jB and rectangular voltages.  With a = |V_i||V_k| cos(t_ik) and
// s = |V_i||V_k| sin(t_ik):
//   dP/dt = G s - B a, dP/dV = (G a + B s)/|V_k|,
//   dQ/dt = -(G a + B s), dQ/dV = (G s - B a)/|V_k|.
// PV rows (|V| equation) and PV columns (fixed |V|) are zeroed.
__device__ __forceinline__ Blk jac_off(double G, double B, double ei, double fi, double ek,
                                       double fk, double vk, bool pv_i, bool pv_k)
{
    double a = ei * ek + fi * fk;
    double s = fi * ek - ei * fk;
    double t1 = G * s - B * a;
    double t2 = G * a + B * s;
    double iv = 1.0 / vk;
    Blk r = {t1, t2 * iv, -t2, t1 * iv};
    if (pv_i) {
        r.c = 0.0;
        r.d = 0.0;
    }
    if (pv_k) {
        r.b = 0.0;
        r.d = 0.0;
    }
    return r;
}

// Diagonal block of bus i from its calculated injection P + jQ:
//   [-Q - B v^2, P/v + G v ; P - G v^2, Q/v - B v];  PV: [-Q - B v^2, 0 ; 0, 1].
__device__ __forceinline__ Blk jac_diag(double G, double B, double P, double Q, double v,
                                        bool pv)
{
    double v2 = v * v;
    if (pv) return {-Q - B * v2, 0.0, 0.0, 1.0};
    double iv = 1.0 / v;
    return {-Q - B * v2, P * iv + G * v, P - G * v2, Q * iv - B * v};
}

}  // namespace pf
