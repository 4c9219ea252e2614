// Internal structures shared by the host analysis and the HIP kernels.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace pf {

// Device view of one symbolic analysis.  Every pointer is a device address
// inside the caller's upload buffer.  Passed to kernels by value, or stored
// in a per-case table for batches with several sparsity patterns.
struct DevSym {
    int32_t n, m, nn, slack;
    int32_t nnz_y, nnz_l, nlev, pad0;
    int64_t n_upd;
    int64_t vals_doubles, ws_doubles;
    // admittance matrix, CSR by bus
    const int32_t* yptr;     // n+1
    const int32_t* ycol;     // nnz_y
    const int32_t* ybr_ptr;  // nnz_y+1: branches contributing to each entry
    const int32_t* ybr;      // ascending branch ids
    // positions
    const int32_t* perm;     // nn: bus at position p
    const int32_t* pos;      // n: position of bus, -1 at the slack
    // filled pattern: S(p) = Li[Lp[p] .. Lp[p+1])
    const int32_t* Lp;       // nn+1
    const int32_t* Li;       // nnz_l
    const int32_t* ylo;      // nnz_l: Y entry (bus k, bus p) for slot (p;k), -1 if fill
    const int32_t* yup;      // nnz_l: Y entry (bus p, bus k), -1 if fill
    const int32_t* ydiag;    // nn: Y entry (bus p, bus p)
    // lower neighbours R(p): descendants i with p in S(i), ascending i
    const int32_t* Rp;       // nn+1
    const int32_t* Ri;       // nnz_l: i
    const int32_t* Rs;       // nnz_l: slot of p in S(i)
    // per destination slot s = (p;k): pairs (slot(i;k), slot(i;p)) of the
    // descendants i that update block (k,p) and (p,k)
    const int32_t* Up;       // nnz_l+1
    const int32_t* Ua;       // n_upd
    const int32_t* Ub;       // n_upd
    // hierarchical partition
    const int32_t* level_ptr;    // nlev+1
    const int32_t* level_nodes;  // nn
    const int32_t* level_g;      // nlev: lanes per node
};

struct HostSym {
    int32_t n = 0, m = 0, nn = 0, slack = 0, ordering = 0;
    std::vector<int32_t> from, to;
    std::vector<int32_t> yptr, ycol, ybr_ptr, ybr;
    std::vector<int32_t> perm, pos, parent, level;
    std::vector<int32_t> Lp, Li, ylo, yup, ydiag;
    std::vector<int32_t> Rp, Ri, Rs;
    std::vector<int32_t> Up, Ua, Ub;
    std::vector<int32_t> level_ptr, level_nodes, level_g;
    int32_t max_width = 0;
    // device copy
    DevSym dev{};
    bool uploaded = false;

    int64_t vals_doubles() const { return 4 * (int64_t)nn + 8 * (int64_t)Li.size(); }
    int64_t ws_doubles() const {
        // vals | e f P Q (n each) | rhs (2 nn)
        int64_t w = vals_doubles() + 4 * (int64_t)n + 2 * (int64_t)nn;
        return (w + 31) & ~(int64_t)31;
    }
    size_t dev_bytes() const;
};

// Host analysis; returns a pf_status code and sets msg on failure.
int analyze(int n, int m, const int32_t* from, const int32_t* to, int slack, int ordering,
            HostSym& out, std::string& msg);
// Default lanes-per-node for every level from a simple work model.
void default_mapping(HostSym& s);

}  // namespace pf
