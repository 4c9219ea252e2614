// libpf C ABI: version and status strings, analysis, symbolic handles
// (info, export, mappings, launch shape, upload) and the shared host helpers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <numeric>
#include <string>
#include <type_traits>
#include <vector>

#include "pf.h"
#include "pf_host.h"
#include "pf_internal.h"

using namespace pf;
using namespace pf::abi;

namespace pf {
namespace abi {

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

int launch_threads(const HostSym& h, int B)
{
    if (h.threads > 0) return h.threads;
    return B <= 512 ? 512 : 256;
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

}  // namespace abi
}  // namespace pf

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
    info->spread = h.spread > 1 ? h.spread : 0;
    info->sub_levels = h.sub_cut;
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
    // every argument is checked before any setting changes
    if (!valid_interleave(interleave))
        return fail(PF_E_INVALID, "pf_symbolic_set_launch: interleave must be 1, 2, 4 or 8");
    if (threads != 0 && threads != 64 && threads != 128 && threads != 256 && threads != 512)
        return fail(PF_E_INVALID, "pf_symbolic_set_launch: threads must be 0, 64, 128, 256 or 512");
    if (tail_lds_budget < 0 || tail_lds_budget > 158 * 1024)
        return fail(PF_E_INVALID, "pf_symbolic_set_launch: tail budget must be 0..161792 bytes");
    s->h.interleave = interleave;
    s->h.threads = threads;
    if (tail_lds_budget != s->h.tail_budget) {
        s->h.tail_budget = tail_lds_budget;
        pf::build_tail(s->h, tail_lds_budget);
        s->h.uploaded = false;  // device copy is stale: upload again
    }
    return PF_OK;
}

int pf_symbolic_set_spread(pf_symbolic s, int workgroups)
{
    if (!s) return fail(PF_E_INVALID, "pf_symbolic_set_spread: NULL symbolic");
    if (workgroups < 0 || workgroups > 1024)
        return fail(PF_E_INVALID, "pf_symbolic_set_spread: workgroups must be 0..1024");
    s->h.spread = workgroups;
    return PF_OK;
}

int pf_symbolic_set_spread_wait(pf_symbolic s, uint64_t ticks)
{
    if (!s) return fail(PF_E_INVALID, "pf_symbolic_set_spread_wait: NULL symbolic");
    s->h.spread_wait = ticks;
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
    // from here on the previous device copy may be overwritten: until this
    // upload succeeds, calls on the symbolic are refused
    h.uploaded = false;
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
    d.sub_cut = h.sub_cut;
    d.sub_roots = h.sub_roots;
    d.sub_idx = put(h.sub_idx);
    d.sub_ptr = put(h.sub_ptr);
    d.sub_cum = put(h.sub_cum);
    s->d_from = put(h.from);
    s->d_to = put(h.to);
    if (off > info.dev_bytes) return fail(PF_E_WORKSPACE, "pf_symbolic_upload: size mismatch");
    int32_t ef_lds = 0;
    {
        int dev = 0, lds_max = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) ==
                hipSuccess) {
            if (h.tail_lds + pv_mask_bytes(h.n) + 2048 > lds_max)
                return fail(PF_E_WORKSPACE, "pf_symbolic_upload: LDS tail larger than the "
                                            "device's LDS; lower it with pf_symbolic_set_launch");
            // the Newton kernel's LDS copy of every bus's (e, f), when it fits
            // the device and the LDS budget the caller set (a small budget
            // leaves room for a second workgroup per CU)
            const int64_t efb = 16 * (int64_t)h.n;
            if (efb + pv_mask_bytes(h.n) + 2048 <= lds_max && efb <= h.tail_budget)
                ef_lds = (int32_t)efb;
        } else {
            (void)hipGetLastError();
        }
        d.ef_lds = ef_lds;
    }
    int rc = hip_check(hipMemcpyAsync(d_buf, stage.data(), off, hipMemcpyHostToDevice,
                                      as_stream(stream)),
                       "pf_symbolic_upload: hipMemcpyAsync");
    if (rc) return rc;
    rc = hip_check(hipStreamSynchronize(as_stream(stream)), "pf_symbolic_upload: sync");
    if (rc) return rc;
    h.ef_lds = ef_lds;
    h.dev = d;
    h.uploaded = true;
    ++h.upload_gen;
    return PF_OK;
}

void pf_symbolic_destroy(pf_symbolic s) { delete s; }

}  // extern "C"
