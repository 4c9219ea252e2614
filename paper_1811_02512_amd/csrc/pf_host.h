// libpf host-side internals shared by the C ABI files: the symbolic handle and
// the argument / error / launch-shape helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "pf.h"
#include "pf_internal.h"

struct pf_symbolic_s {
    pf::HostSym h;
    const int32_t* d_from = nullptr;  // device copies of the branch ends
    const int32_t* d_to = nullptr;
};

namespace pf {
namespace abi {

// Thread-local message of the last failed call (pf_last_error).
extern thread_local std::string g_err;

// Records msg as the thread's last error and returns code.
int fail(int code, const std::string& msg);
int hip_check(hipError_t e, const char* what);
int launch_check(const char* what);
// Workgroup size of the level-scheduled kernels: the symbolic's setting, or
// by batch size.
int launch_threads(const pf::HostSym& h, int B);
// Blocks for B cases in groups of C placed one XCD round apart.
int grid_blocks(int B, int C);
bool valid_interleave(int C);
// Interleave pf_newton uses for B cases.
int newton_interleave(const pf::HostSym& h, int B);
// A symbolic that is non-null and uploaded (else records the error).
bool ready(const pf_symbolic s, const char* fn);
inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }
// A per-case stride of an input that the cases may also share: 0 (one array
// for all cases) or, with more than one case, at least one row.
inline bool shared_stride_ok(int B, int64_t stride, int64_t row)
{
    return stride >= 0 && (stride == 0 || B <= 1 || stride >= row);
}
// Branch gradients (and, with bus, the injection gradients) of B cases from
// their adjoint vectors (pf_adjoint_params, pf_adjoint).
int adjoint_branch_launch(const pf_symbolic s, int B, const double* d_lam, int64_t lam_stride,
                          const int8_t* d_type, int64_t type_stride, const double* d_Vm,
                          const double* d_Va, int64_t v_stride, const double* d_r,
                          const double* d_x, int64_t branch_stride, const int32_t* d_status,
                          double* d_gP, double* d_gQ, int64_t g_stride, double* d_gx,
                          int gx_mode, void* stream, bool bus);
// The level-scheduled factorisation of B matrices (sym: symmetric ones).
void factor_launch(const pf::HostSym& h, int B, double* vals, int64_t stride, int C,
                   int32_t* status, int32_t* pivot, hipStream_t st, bool sym);

}  // namespace abi
}  // namespace pf
