// Internal structures shared by the host analysis and the HIP kernels.
#pragma once

#include <hip/hip_vector_types.h>

#include <cstdint>
#include <string>
#include <vector>

namespace pf {

// Device view of one symbolic analysis.  Every pointer is a device address
// inside the caller's upload buffer.  Passed to kernels by value, or stored
// in a per-case table for batches with several sparsity patterns.
//
// Packed records (int4 = 4 x int32) let a lane fetch everything it needs
// about a node or a slot with one or two wide loads instead of a chain of
// dependent scalar loads:
//   node_info[x] (level order, 3 x int4): {j, bus, r0, r1}, {s0, s1, ydiag, 0},
//                                          {q0, q1, 0, 0}
//     j = position, [r0, r1) = its lower-neighbour range in rl,
//     [s0, s1) = its slots (higher neighbours), ydiag = Y entry (bus, bus),
//     [q0, q1) = the bus's admittance row
//   slot_info[s] (2 x int4): {k, bus_k, ylo, yup}, {u0, u1, 0, 0}
//     k = higher neighbour, ylo/yup = Y entries (bus_k, bus_j) / (bus_j,
//     bus_k) or -1 for fill, [u0, u1) = its update pairs in upd
//   rl[r] = (i, slot(i;j))      upd[u] = (slot(i;k), slot(i;j))
//
// Tail: the top levels [tail_level, nlev) of the elimination tree, whose
// values fit in LDS, are factorised and solved in LDS.  Every higher
// neighbour of a tail node is itself in the tail.  Local numbering: tail
// nodes 0..K-1 in level order, tail slots 0..TS-1 in node order.
//   t_node[jl] (3 x int4): {j, bus, ydiag, sl0}, {sl1, rn0, rn1, rt1}, {rmid, pk, 0, 0}
//     [sl0, sl1) local slots, [rn0, rn1) lower neighbours outside the tail
//     as (i, slot) global pairs in t_rl, [rn1, rt1) lower neighbours inside
//     the tail as (local i, local slot) pairs in t_rl, those below the
//     clique first: [rn1, rmid) below, [rmid, rt1) in the clique
//   t_slot[t] (3 x int4): {s, kl, bus_k, ylo}, {yup, un0, un1, ut1},
//                         {bus_j, jl, umid, pk}
//     s = global slot, kl = local node of k, [un0, un1) update pairs from
//     outside the tail (global slots) and [un1, ut1) from inside (local),
//     [un1, umid) from below the clique, [umid, ut1) from the clique;
//     jl = local node owning the slot
//   The clique is the last tail_clique local nodes: a chain of single-node
//   levels, each adjacent to every node above it (local slot of clique pair
//   (a, b), a < b, is t_node[a].sl0 + b - a - 1).
//   t_lptr[l - tail_level .. ]: local node range of each tail level
//   t_pk: the local lists again, packed: each 32-bit word holds a local pair
//     (lo 16 bits, hi 16 bits), four words per 16-byte load; a node's local
//     lower neighbours [rn1, rt1) start at load t_node.pk, a slot's local
//     update pairs [un1, ut1) at load t_slot.pk; each list is padded to
//     whole loads
struct DevSym {
    int32_t n, m, nn, slack;
    int32_t nnz_y, nnz_l, nlev, pad0;
    int64_t n_upd;
    int64_t vals_doubles, ws_doubles;
    int64_t lu_off;  // doubles before the LU section (D padded to 64 bytes)
    int64_t fd_lu, fd_mat;  // fast decoupled: d section (padded), one matrix
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
    // hierarchical partition
    const int32_t* level_ptr;    // nlev+1
    const int32_t* level_nodes;  // nn
    const int32_t* level_g;      // nlev: lanes per node
    // packed records
    const int4* node_info;   // 3 nn
    const int4* slot_info;   // 2 nnz_l
    const int2* rl;          // nnz_l
    const int2* upd;         // n_upd
    // LDS tail
    int32_t tail_level, tail_nodes, tail_slots, tail_lds;
    int32_t tail_clique;
    int32_t ef_lds;  // bytes of the LDS copy of (e, f) per bus the Newton mismatch reads, 0 = none
    const int4* t_node;      // 3 K
    const int4* t_slot;      // 3 TS
    const int2* t_rl;
    const int2* t_upd;
    const int32_t* t_lptr;   // nlev - tail_level + 1
    const uint4* t_pk;
    // Subtrees below a cut level (the group of workgroups that a spread
    // batch of grids gives a case hands each workgroup whole subtrees there,
    // so those levels need workgroup barriers only; a one-case spread launch
    // shares them and does not read these tables).  Roots: nodes of levels [0, sub_cut)
    // whose parent lies at level sub_cut or above (or is absent), numbered
    // by position.
    //   sub_idx[x] for x < level_ptr[sub_cut]: the level-ordered node
    //     records of each level again, grouped by root (ascending root,
    //     then record)
    //   sub_ptr[l (sub_roots + 1) + k]: entries of level l's group whose
    //     root is below k
    //   sub_cum[k]: work of the subtrees of roots below k (sub_roots + 1)
    int32_t sub_cut, sub_roots;
    const int32_t* sub_idx;
    const int32_t* sub_ptr;
    const int32_t* sub_cum;
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
    std::vector<int32_t> node_info, slot_info, rl, upd;  // packed (int32 view)
    // tail
    int32_t tail_level = 0, tail_nodes = 0, tail_slots = 0, tail_lds = 0, tail_clique = 0;
    int64_t tail_budget = 64 * 1024;
    std::vector<int32_t> t_node, t_slot, t_rl, t_upd, t_lptr, t_pk;
    // subtrees below a cut level (DevSym); rebuilt with the tail
    int32_t sub_cut = 0, sub_roots = 0;
    std::vector<int32_t> sub_idx, sub_ptr, sub_cum;
    int32_t ef_lds = 0;  // set at upload: 16 n when it fits in the device's LDS, else 0
    int32_t max_width = 0;
    int32_t threads = 0;  // 0: chosen per launch from the batch size
    int32_t interleave = 4;  // cases per interleaved workspace group
    // workgroups a one-case Newton launch spreads its wide phases over (the
    // bus loops and the levels below the LDS tail); 0 or 1: one workgroup
    int32_t spread = 0;
    // longest wait at a grid barrier of a spread launch, in ticks of the
    // 100 MHz constant clock, before the launch gives up (one second)
    uint64_t spread_wait = 100000000ull;
    // device copy
    DevSym dev{};
    bool uploaded = false;
    // counts uploads; a batch plan built over this symbolic records it and
    // refuses to run once the device copy has been replaced or gone stale
    uint64_t upload_gen = 0;

    // D [nn][4], zero padding to a multiple of 8 doubles, LU [nnz_l][8]: every
    // slot record (W, U) and bus record starts on a 64-byte boundary.
    int64_t lu_off() const { return 8 * (((int64_t)nn + 1) / 2); }
    int64_t vals_doubles() const { return lu_off() + 8 * (int64_t)Li.size(); }
    // fast decoupled matrices: per matrix d [fd_lu()] | (w, u) per slot; two
    // matrices (B', B'') per case
    int64_t fd_lu() const { return ((int64_t)nn + 7) & ~(int64_t)7; }
    int64_t fd_mat() const { return (fd_lu() + 2 * (int64_t)Li.size() + 7) & ~(int64_t)7; }
    int64_t fd_ws_doubles() const {
        int64_t w = 8 * (int64_t)n + 2 * (int64_t)nn;  // bus records | rhs
        return (w + 31) & ~(int64_t)31;
    }
    // vals | bus records (8 n) | rhs (2 nn) | grid-barrier words of a one-case
    // launch spread over several workgroups (three 128-byte lines)
    int64_t sync_off() const {
        return (vals_doubles() + 8 * (int64_t)n + 2 * (int64_t)nn + 15) & ~(int64_t)15;
    }
    int64_t ws_doubles() const { return (sync_off() + 48 + 31) & ~(int64_t)31; }
    size_t dev_bytes() const;
};

// LDS bytes of a tail with K nodes and TS slots: W and U (or V) blocks per
// slot, D^-1 and the forward vector per node.
inline int64_t tail_bytes(int64_t K, int64_t TS) { return TS * 64 + K * 48; }

// LDS bytes of the PV bitmask the Newton kernel keeps after the tail (one bit
// per bus, whole 64-bit ballot words).
inline int64_t pv_mask_bytes(int64_t n) { return 8 * ((n + 63) / 64); }

// Host analysis; returns a pf_status code and sets msg on failure.
int analyze(int n, int m, const int32_t* from, const int32_t* to, int slack, int ordering,
            HostSym& out, std::string& msg);
// Default lanes-per-node for every level from a simple work model.
void default_mapping(HostSym& s);
// (Re)builds the LDS tail for an LDS budget in bytes (0 disables it), and
// the subtrees below the cut level under it.
void build_tail(HostSym& s, int64_t budget);
// Subtrees of the levels below the tail for spread launches: the highest cut
// at or below the tail level with at least kSubMinRoots roots (none if no
// such level).
constexpr int kSubMinRoots = 768;
void build_subtrees(HostSym& s);

}  // namespace pf
