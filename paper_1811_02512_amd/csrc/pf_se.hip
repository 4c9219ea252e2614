// libpf WLS state estimation (device code, kernels, host plan and C ABI).
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
                   const double* d_b, int64_t branch_stride, const double* d_ysh,
                   int64_t ysh_stride, const double* d_z,
                   int64_t z_stride, const double* d_w, int64_t w_stride, double* d_Vm,
                   double* d_Va, int64_t v_stride, double tol, int max_iter, double* d_ws,
                   int64_t ws_size, int32_t* d_iters, double* d_norm, int32_t* d_status,
                   void* stream)
{
    if (!s || !s->uploaded) return fail(PF_E_INVALID, "pf_se_estimate: not uploaded");
    if (B < 0 || B > 65535 || max_iter < 1 || !(tol >= 0.0) || !d_r || !d_x || !d_b || !d_z ||
        !d_w || !d_Vm || !d_Va || !d_ws || !d_iters || !d_norm || !d_status || z_stride < 0 ||
        w_stride < 0 || branch_stride < 0 || ysh_stride < 0)
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
    // admittance copies: one per case when the branches or the shunts differ
    const bool per_case_y = branch_stride != 0 || (d_ysh && ysh_stride != 0);
    const int yb = per_case_y ? B : 1;
    SeWs X;
    X.B = B;
    X.C = kSeGroup;
    X.vals = d_ws;
    X.vs = s->vs;
    X.rhs = X.vals + (int64_t)Bg * s->vs;
    X.rs = s->rs;
    X.y = X.rhs + (int64_t)B * s->rs;
    X.ys = per_case_y ? s->ys : 0;
    X.st = reinterpret_cast<double2*>(X.y + (int64_t)yb * s->ys);
    X.par = X.st + 2 * (int64_t)s->n * B;
    X.res = reinterpret_cast<double*>(X.par + s->P * B);
    hipLaunchKernelGGL(k_se_start, dim3((B + 255) / 256), dim3(256), 0, st, B, d_iters, d_norm,
                       d_status);
    int rc = launch_check("pf_se_estimate: start");
    if (rc) return rc;
    rc = pf_build_ybus(&s->net, yb, d_r, d_x, d_b, branch_stride, d_ysh, ysh_stride, X.y, s->ys,
                       stream);
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
        factor_launch(G, B, X.vals, X.vs, kSeGroup, nullptr, nullptr, st, true);
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
