// Host symbolic analysis for the level-scheduled block LDU.
//
// Steps (paper, Sec. II-B): fill-reducing elimination order (our reading:
// exact minimum degree, the paper itself eliminates in the given numbering),
// FormFilledGraph, FormEliminationTree, FormHierarchicalPartition.  The
// filled pattern falls out of the symbolic elimination itself: the neighbours
// a node still has when it is eliminated are exactly its higher neighbours in
// the filled graph.  On top of the paper's structures this builds the index
// maps the kernels need: admittance CSR with its contributing branches,
// position <-> bus maps, Y entry of every filled block, lower-neighbour lists
// and the per-destination update pairs of the left-looking factorisation.
#include <algorithm>
#include <cstring>
#include <queue>
#include <utility>

#include "pf.h"
#include "pf_internal.h"

namespace pf {

namespace {

// Sorted-vector union of a and b without the values x and y.
void merge_without(const std::vector<int32_t>& a, const std::vector<int32_t>& b, int32_t x,
                   int32_t y, std::vector<int32_t>& out)
{
    out.clear();
    out.reserve(a.size() + b.size());
    size_t i = 0, j = 0;
    while (i < a.size() || j < b.size()) {
        int32_t v;
        if (j >= b.size() || (i < a.size() && a[i] < b[j])) {
            v = a[i++];
        } else if (i >= a.size() || b[j] < a[i]) {
            v = b[j++];
        } else {
            v = a[i++];
            ++j;
        }
        if (v != x && v != y) out.push_back(v);
    }
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

size_t HostSym::dev_bytes() const
{
    const std::vector<int32_t>* arrs[] = {&yptr,      &ycol,      &ybr_ptr, &ybr,    &perm,
                                          &pos,       &Lp,        &Li,      &ylo,    &yup,
                                          &ydiag,     &Rp,        &Ri,      &Rs,     &level_ptr,
                                          &level_nodes, &level_g, &node_info, &slot_info, &rl,
                                          &upd,       &t_node,    &t_slot,  &t_rl,   &t_upd,
                                          &t_lptr,    &t_pk,      &from,    &to,     &sub_idx,
                                          &sub_ptr,   &sub_cum};
    size_t total = 0;
    for (auto* a : arrs) total += align256(std::max<size_t>(a->size(), 1) * sizeof(int32_t));
    return total;
}

int analyze(int n, int m, const int32_t* from, const int32_t* to, int slack, int ordering,
            HostSym& s, std::string& msg)
{
    if (n < 2 || m < 0 || slack < 0 || slack >= n || (m > 0 && (!from || !to))) {
        msg = "pf_analyze: need n >= 2, m >= 0, 0 <= slack < n and branch arrays";
        return PF_E_INVALID;
    }
    if (ordering != PF_ORDER_MINDEG && ordering != PF_ORDER_NATURAL) {
        msg = "pf_analyze: unknown ordering";
        return PF_E_INVALID;
    }
    for (int e = 0; e < m; ++e) {
        if (from[e] < 0 || from[e] >= n || to[e] < 0 || to[e] >= n) {
            msg = "pf_analyze: branch " + std::to_string(e) + " has a bus index out of range";
            return PF_E_INVALID;
        }
        if (from[e] == to[e]) {
            msg = "pf_analyze: branch " + std::to_string(e) + " is a self loop";
            return PF_E_INVALID;
        }
    }
    s = HostSym();
    s.n = n;
    s.m = m;
    s.nn = n - 1;
    s.slack = slack;
    s.ordering = ordering;
    s.from.assign(from, from + m);
    s.to.assign(to, to + m);

    // incidence: (other bus, branch) per bus, sorted
    std::vector<std::vector<std::pair<int32_t, int32_t>>> inc(n);
    for (int e = 0; e < m; ++e) {
        inc[from[e]].push_back({to[e], e});
        inc[to[e]].push_back({from[e], e});
    }
    for (auto& v : inc) std::sort(v.begin(), v.end());

    // every bus must reach the slack
    {
        std::vector<char> seen(n, 0);
        std::vector<int32_t> stack{slack};
        seen[slack] = 1;
        int cnt = 1;
        while (!stack.empty()) {
            int v = stack.back();
            stack.pop_back();
            for (auto& pe : inc[v])
                if (!seen[pe.first]) {
                    seen[pe.first] = 1;
                    ++cnt;
                    stack.push_back(pe.first);
                }
        }
        if (cnt != n) {
            msg = "pf_analyze: " + std::to_string(n - cnt) + " bus(es) not connected to the slack";
            return PF_E_DISCONNECTED;
        }
    }

    // admittance CSR (diagonal always present) and contributing branches
    s.yptr.assign(n + 1, 0);
    s.ybr_ptr.push_back(0);
    for (int i = 0; i < n; ++i) {
        std::vector<int32_t> cols;
        cols.push_back(i);
        for (auto& pe : inc[i]) cols.push_back(pe.first);
        std::sort(cols.begin(), cols.end());
        cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
        for (int32_t c : cols) {
            s.ycol.push_back(c);
            if (c == i) {
                std::vector<int32_t> br;
                for (auto& pe : inc[i]) br.push_back(pe.second);
                std::sort(br.begin(), br.end());
                s.ybr.insert(s.ybr.end(), br.begin(), br.end());
            } else {
                for (auto& pe : inc[i])
                    if (pe.first == c) s.ybr.push_back(pe.second);  // ascending branch id
            }
            s.ybr_ptr.push_back((int32_t)s.ybr.size());
        }
        s.yptr[i + 1] = (int32_t)s.ycol.size();
    }
    auto yfind = [&](int32_t row, int32_t col) -> int32_t {
        auto b = s.ycol.begin() + s.yptr[row], e = s.ycol.begin() + s.yptr[row + 1];
        auto it = std::lower_bound(b, e, col);
        return (it != e && *it == col) ? (int32_t)(it - s.ycol.begin()) : -1;
    };

    // reduced graph: node v <-> bus, ascending bus order without the slack
    const int nn = s.nn;
    std::vector<int32_t> bus_of(nn), node_of(n, -1);
    for (int i = 0, v = 0; i < n; ++i)
        if (i != slack) {
            node_of[i] = v;
            bus_of[v++] = i;
        }
    std::vector<std::vector<int32_t>> adj(nn);
    for (int v = 0; v < nn; ++v) {
        int i = bus_of[v];
        for (auto& pe : inc[i]) {
            int w = node_of[pe.first];
            if (w >= 0) adj[v].push_back(w);
        }
        std::sort(adj[v].begin(), adj[v].end());
        adj[v].erase(std::unique(adj[v].begin(), adj[v].end()), adj[v].end());
    }

    // symbolic elimination: minimum degree (ties to the lowest node, i.e.
    // lowest bus) or the natural order; hi[v] = neighbours left at elimination
    std::vector<std::vector<int32_t>> hi(nn);
    std::vector<int32_t> order(nn);
    {
        std::vector<char> gone(nn, 0);
        using Item = std::pair<int32_t, int32_t>;  // (degree, node)
        std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
        if (ordering == PF_ORDER_MINDEG)
            for (int v = 0; v < nn; ++v) heap.push({(int32_t)adj[v].size(), v});
        std::vector<int32_t> tmp;
        for (int step = 0; step < nn; ++step) {
            int p;
            if (ordering == PF_ORDER_NATURAL) {
                p = step;
            } else {
                for (;;) {
                    Item it = heap.top();
                    heap.pop();
                    if (!gone[it.second] && it.first == (int32_t)adj[it.second].size()) {
                        p = it.second;
                        break;
                    }
                }
            }
            order[step] = p;
            gone[p] = 1;
            hi[p] = adj[p];
            for (int32_t a : hi[p]) {
                merge_without(adj[a], hi[p], a, p, tmp);
                adj[a].swap(tmp);
                if (ordering == PF_ORDER_MINDEG) heap.push({(int32_t)adj[a].size(), a});
            }
            adj[p].clear();
            adj[p].shrink_to_fit();
        }
    }

    // positions and the filled pattern S(p)
    std::vector<int32_t> pos_of_node(nn);
    for (int p = 0; p < nn; ++p) pos_of_node[order[p]] = p;
    s.perm.resize(nn);
    s.pos.assign(n, -1);
    for (int p = 0; p < nn; ++p) {
        s.perm[p] = bus_of[order[p]];
        s.pos[s.perm[p]] = p;
    }
    s.Lp.assign(nn + 1, 0);
    for (int p = 0; p < nn; ++p) {
        std::vector<int32_t> sp;
        for (int32_t v : hi[order[p]]) sp.push_back(pos_of_node[v]);
        std::sort(sp.begin(), sp.end());
        s.Li.insert(s.Li.end(), sp.begin(), sp.end());
        s.Lp[p + 1] = (int32_t)s.Li.size();
    }
    hi.clear();
    const int64_t nnzl = (int64_t)s.Li.size();

    // elimination tree and levels (level = 1 + highest child level)
    s.parent.assign(nn, -1);
    s.level.assign(nn, 1);
    for (int p = 0; p < nn; ++p) {
        if (s.Lp[p + 1] > s.Lp[p]) s.parent[p] = s.Li[s.Lp[p]];
        if (s.parent[p] >= 0)
            s.level[s.parent[p]] = std::max(s.level[s.parent[p]], s.level[p] + 1);
    }
    int nlev = 0;
    for (int p = 0; p < nn; ++p) nlev = std::max(nlev, s.level[p]);
    s.level_ptr.assign(nlev + 1, 0);
    for (int p = 0; p < nn; ++p) s.level_ptr[s.level[p]]++;
    for (int l = 0; l < nlev; ++l) s.level_ptr[l + 1] += s.level_ptr[l];
    s.level_nodes.assign(nn, 0);
    {
        std::vector<int32_t> cur(s.level_ptr.begin(), s.level_ptr.end() - 1);
        for (int p = 0; p < nn; ++p) s.level_nodes[cur[s.level[p] - 1]++] = p;
    }
    s.max_width = 0;
    for (int l = 0; l < nlev; ++l)
        s.max_width = std::max(s.max_width, s.level_ptr[l + 1] - s.level_ptr[l]);

    // admittance entries of every block
    s.ydiag.resize(nn);
    s.ylo.resize(nnzl);
    s.yup.resize(nnzl);
    for (int p = 0; p < nn; ++p) {
        int bp = s.perm[p];
        s.ydiag[p] = yfind(bp, bp);
        for (int q = s.Lp[p]; q < s.Lp[p + 1]; ++q) {
            int bk = s.perm[s.Li[q]];
            s.ylo[q] = yfind(bk, bp);
            s.yup[q] = yfind(bp, bk);
        }
    }

    // lower neighbours R(p) with the slot of p inside S(i), ascending i
    s.Rp.assign(nn + 1, 0);
    for (int64_t q = 0; q < nnzl; ++q) s.Rp[s.Li[q] + 1]++;
    for (int p = 0; p < nn; ++p) s.Rp[p + 1] += s.Rp[p];
    s.Ri.resize(nnzl);
    s.Rs.resize(nnzl);
    {
        std::vector<int32_t> cur(s.Rp.begin(), s.Rp.end() - 1);
        for (int i = 0; i < nn; ++i)
            for (int q = s.Lp[i]; q < s.Lp[i + 1]; ++q) {
                int k = s.Li[q];
                s.Ri[cur[k]] = i;
                s.Rs[cur[k]] = q;
                cur[k]++;
            }
    }

    // update pairs per destination slot.  For node j and descendant i with
    // b = slot(i;j), every k after j in S(i) is also in S(j) (the higher
    // neighbours of a node form a clique in the filled graph); the block
    // pair at a = slot(i;k) updates destination slot(j;k).
    s.Up.assign(nnzl + 1, 0);
    for (int pass = 0; pass < 2; ++pass) {
        std::vector<int32_t> cur;
        if (pass == 1) {
            for (int64_t q = 0; q < nnzl; ++q) s.Up[q + 1] += s.Up[q];
            s.Ua.resize(s.Up[nnzl]);
            s.Ub.resize(s.Up[nnzl]);
            cur.assign(s.Up.begin(), s.Up.end() - 1);
        }
        for (int j = 0; j < nn; ++j) {
            for (int r = s.Rp[j]; r < s.Rp[j + 1]; ++r) {
                int i = s.Ri[r], b = s.Rs[r];
                int d = s.Lp[j];
                for (int a = b + 1; a < s.Lp[i + 1]; ++a) {
                    int k = s.Li[a];
                    while (d < s.Lp[j + 1] && s.Li[d] < k) ++d;
                    if (d >= s.Lp[j + 1] || s.Li[d] != k) {
                        msg = "pf_analyze: internal error, filled pattern is not closed";
                        return PF_E_INVALID;
                    }
                    if (pass == 0) {
                        s.Up[d + 1]++;
                    } else {
                        s.Ua[cur[d]] = a;
                        s.Ub[cur[d]] = b;
                        cur[d]++;
                    }
                }
            }
        }
    }

    // packed records (layouts documented with DevSym)
    s.node_info.assign(12 * (size_t)nn, 0);
    for (int x = 0; x < nn; ++x) {
        const int j = s.level_nodes[x];
        int32_t* r = &s.node_info[12 * (size_t)x];
        r[0] = j;
        r[1] = s.perm[j];
        r[2] = s.Rp[j];
        r[3] = s.Rp[j + 1];
        r[4] = s.Lp[j];
        r[5] = s.Lp[j + 1];
        r[6] = s.ydiag[j];
        r[8] = s.yptr[s.perm[j]];
        r[9] = s.yptr[s.perm[j] + 1];
    }
    s.slot_info.assign(8 * (size_t)nnzl, 0);
    for (int64_t q = 0; q < nnzl; ++q) {
        int32_t* r = &s.slot_info[8 * (size_t)q];
        r[0] = s.Li[q];
        r[1] = s.perm[s.Li[q]];
        r[2] = s.ylo[q];
        r[3] = s.yup[q];
        r[4] = s.Up[q];
        r[5] = s.Up[q + 1];
    }
    s.rl.resize(2 * (size_t)nnzl);
    for (int64_t q = 0; q < nnzl; ++q) {
        s.rl[2 * q] = s.Ri[q];
        s.rl[2 * q + 1] = s.Rs[q];
    }
    s.upd.resize(2 * s.Ua.size());
    for (size_t u = 0; u < s.Ua.size(); ++u) {
        s.upd[2 * u] = s.Ua[u];
        s.upd[2 * u + 1] = s.Ub[u];
    }
    default_mapping(s);
    build_tail(s, s.tail_budget);
    return PF_OK;
}

// The LDS tail: the largest run of top levels whose values, with the
// Newton kernel's PV bitmask, fit the budget.
// Its top may be a clique chain: single-node levels where every node is
// adjacent to all nodes above it in the filled graph.  That part is
// factorised and solved densely (right-looking, one barrier per pivot).
void build_tail(HostSym& s, int64_t budget)
{
    const int nlev = (int)s.level_ptr.size() - 1;
    const int nn = s.nn;
    int L = nlev;
    int64_t K = 0, TS = 0;
    if (budget > 0) {
        while (L > 0) {
            const int l = L - 1;
            int64_t k2 = K, t2 = TS;
            for (int x = s.level_ptr[l]; x < s.level_ptr[l + 1]; ++x) {
                const int j = s.level_nodes[x];
                ++k2;
                t2 += s.Lp[j + 1] - s.Lp[j];
            }
            if (tail_bytes(k2, t2) + pv_mask_bytes(s.n) > budget || t2 > 65535) break;
            K = k2;
            TS = t2;
            L = l;
        }
    }
    s.tail_level = L;
    s.tail_nodes = (int32_t)K;
    s.tail_slots = (int32_t)TS;
    s.tail_lds = K ? (int32_t)tail_bytes(K, TS) : 0;
    s.tail_clique = 0;
    s.t_node.clear();
    s.t_slot.clear();
    s.t_rl.clear();
    s.t_upd.clear();
    s.t_pk.clear();
    s.t_lptr.assign(1, 0);
    build_subtrees(s);
    if (K == 0) return;

    // clique chain at the top of the tail: level nlev-1-d holds one node
    // whose higher neighbours are exactly the d chain nodes above it
    {
        std::vector<int32_t> chain;  // from the root down
        for (int l = nlev - 1; l >= L; --l) {
            if (s.level_ptr[l + 1] - s.level_ptr[l] != 1) break;
            const int j = s.level_nodes[s.level_ptr[l]];
            const int d = (int)chain.size();
            if (s.Lp[j + 1] - s.Lp[j] != d) break;
            bool ok = true;
            for (int q = 0; q < d && ok; ++q) ok = s.Li[s.Lp[j] + q] == chain[d - 1 - q];
            if (!ok) break;
            chain.push_back(j);
        }
        s.tail_clique = chain.size() >= 3 ? (int32_t)chain.size() : 0;
    }

    const int64_t nnzl = (int64_t)s.Li.size();
    std::vector<int32_t> loc(nn, -1), sloc(nnzl, -1), owner(nnzl, -1);
    for (int p = 0; p < nn; ++p)
        for (int q = s.Lp[p]; q < s.Lp[p + 1]; ++q) owner[q] = p;
    std::vector<int32_t> tnodes;
    for (int l = L; l < nlev; ++l) {
        for (int x = s.level_ptr[l]; x < s.level_ptr[l + 1]; ++x) {
            loc[s.level_nodes[x]] = (int32_t)tnodes.size();
            tnodes.push_back(s.level_nodes[x]);
        }
        s.t_lptr.push_back((int32_t)tnodes.size());
    }
    const int32_t kfirst = (int32_t)K - s.tail_clique;  // first local node of the clique
    auto in_clique = [&](int p) { return loc[p] >= kfirst; };
    int32_t ts = 0;
    for (int j : tnodes)
        for (int q = s.Lp[j]; q < s.Lp[j + 1]; ++q) sloc[q] = ts++;
    s.t_node.assign(12 * (size_t)K, 0);
    s.t_slot.assign(12 * (size_t)TS, 0);
    int32_t run = 0;
    for (size_t jl = 0; jl < tnodes.size(); ++jl) {
        const int j = tnodes[jl];
        int32_t* r = &s.t_node[12 * jl];
        r[0] = j;
        r[1] = s.perm[j];
        r[2] = s.ydiag[j];
        r[3] = run;  // local slots were numbered in this same node order
        run += s.Lp[j + 1] - s.Lp[j];
        r[4] = run;
        r[5] = (int32_t)(s.t_rl.size() / 2);
        for (int q = s.Rp[j]; q < s.Rp[j + 1]; ++q)
            if (loc[s.Ri[q]] < 0) {
                s.t_rl.push_back(s.Ri[q]);
                s.t_rl.push_back(s.Rs[q]);
            }
        r[6] = (int32_t)(s.t_rl.size() / 2);
        for (int pass = 0; pass < 2; ++pass) {  // tail descendants below the clique first
            for (int q = s.Rp[j]; q < s.Rp[j + 1]; ++q) {
                const int i = s.Ri[q];
                if (loc[i] >= 0 && in_clique(i) == (pass == 1)) {
                    s.t_rl.push_back(loc[i]);
                    s.t_rl.push_back(sloc[s.Rs[q]]);
                }
            }
            if (pass == 0) r[8] = (int32_t)(s.t_rl.size() / 2);
        }
        r[7] = (int32_t)(s.t_rl.size() / 2);
        for (int q = s.Lp[j]; q < s.Lp[j + 1]; ++q) {
            int32_t* t = &s.t_slot[12 * (size_t)sloc[q]];
            t[0] = q;
            t[1] = loc[s.Li[q]];
            t[2] = s.perm[s.Li[q]];
            t[3] = s.ylo[q];
            t[4] = s.yup[q];
            t[5] = (int32_t)(s.t_upd.size() / 2);
            for (int u = s.Up[q]; u < s.Up[q + 1]; ++u)
                if (loc[owner[s.Ub[u]]] < 0) {
                    s.t_upd.push_back(s.Ua[u]);
                    s.t_upd.push_back(s.Ub[u]);
                }
            t[6] = (int32_t)(s.t_upd.size() / 2);
            for (int pass = 0; pass < 2; ++pass) {
                for (int u = s.Up[q]; u < s.Up[q + 1]; ++u) {
                    const int i = owner[s.Ub[u]];
                    if (loc[i] >= 0 && in_clique(i) == (pass == 1)) {
                        s.t_upd.push_back(sloc[s.Ua[u]]);
                        s.t_upd.push_back(sloc[s.Ub[u]]);
                    }
                }
                if (pass == 0) t[10] = (int32_t)(s.t_upd.size() / 2);
            }
            t[7] = (int32_t)(s.t_upd.size() / 2);
            t[8] = s.perm[j];
            t[9] = (int32_t)jl;
        }
    }
    // packed copies of the local lists (local indices are below 2^16: the
    // tail's slots fit in LDS)
    auto pack = [&](const std::vector<int32_t>& src, int32_t b, int32_t e) {
        const int32_t start = (int32_t)(s.t_pk.size() / 4);
        for (int32_t u = b; u < e; ++u)
            s.t_pk.push_back((int32_t)((uint32_t)src[2 * (size_t)u] |
                                       ((uint32_t)src[2 * (size_t)u + 1] << 16)));
        while (s.t_pk.size() % 4) s.t_pk.push_back(0);
        return start;
    };
    for (int64_t jl = 0; jl < K; ++jl) {
        int32_t* r = &s.t_node[12 * (size_t)jl];
        r[9] = pack(s.t_rl, r[6], r[7]);
    }
    for (int64_t t = 0; t < TS; ++t) {
        int32_t* u = &s.t_slot[12 * (size_t)t];
        u[11] = pack(s.t_upd, u[6], u[7]);
    }
}

void build_subtrees(HostSym& s)
{
    const int nlev = (int)s.level_ptr.size() - 1;
    const int nn = s.nn;
    s.sub_cut = 0;
    s.sub_roots = 0;
    s.sub_idx.clear();
    s.sub_ptr.clear();
    s.sub_cum.clear();
    const int top = std::min(s.tail_level, nlev);
    if (top <= 0 || nn == 0) return;
    // roots below cut c (levels 0-based here): nodes p with level(p) < c
    // <= level(parent(p)), or without a parent; counted for every c at once
    std::vector<int64_t> diff(nlev + 2, 0);
    for (int p = 0; p < nn; ++p) {
        const int lp = s.level[p] - 1;
        const int hi = s.parent[p] >= 0 ? s.level[s.parent[p]] - 1 : nlev;
        diff[lp + 1] += 1;
        diff[hi + 1] -= 1;
    }
    int cut = 0;
    int64_t run = 0;
    for (int c = 1; c <= top; ++c) {
        run += diff[c];
        if (run >= kSubMinRoots) cut = c;
    }
    if (cut == 0) return;
    // each node's root (its parent is on a higher level, so top-down works)
    std::vector<int32_t> root(nn, -1);
    for (int l = cut - 1; l >= 0; --l)
        for (int x = s.level_ptr[l]; x < s.level_ptr[l + 1]; ++x) {
            const int p = s.level_nodes[x];
            const int q = s.parent[p];
            root[p] = (q < 0 || s.level[q] - 1 >= cut) ? p : root[q];
        }
    std::vector<int32_t> rid(nn, -1);
    int32_t R = 0;
    for (int p = 0; p < nn; ++p)
        if (root[p] == p) rid[p] = R++;
    // work of a node: its record, descendant list and slots with their pairs
    std::vector<int64_t> W(R, 0);
    for (int p = 0; p < nn; ++p) {
        if (root[p] < 0) continue;
        int64_t w = 4 + (s.Rp[p + 1] - s.Rp[p]);
        for (int q = s.Lp[p]; q < s.Lp[p + 1]; ++q) w += 2 + (s.Up[q + 1] - s.Up[q]);
        W[rid[root[p]]] += w;
    }
    int64_t tot = 0;
    for (int64_t w : W) tot += w;
    if (tot >= ((int64_t)1 << 30)) return;
    s.sub_cum.assign(R + 1, 0);
    for (int k = 0; k < R; ++k) s.sub_cum[k + 1] = s.sub_cum[k] + (int32_t)W[k];
    s.sub_idx.resize(s.level_ptr[cut]);
    s.sub_ptr.assign((size_t)cut * (R + 1), 0);
    for (int l = 0; l < cut; ++l) {
        const int b = s.level_ptr[l], e = s.level_ptr[l + 1];
        std::vector<int32_t> xs(e - b);
        for (int x = b; x < e; ++x) xs[x - b] = x;
        std::stable_sort(xs.begin(), xs.end(), [&](int32_t u, int32_t v) {
            return rid[root[s.level_nodes[u]]] < rid[root[s.level_nodes[v]]];
        });
        int32_t* ptr = &s.sub_ptr[(size_t)l * (R + 1)];
        for (int i = 0; i < e - b; ++i) {
            s.sub_idx[b + i] = xs[i];
            ++ptr[rid[root[s.level_nodes[xs[i]]]] + 1];
        }
        for (int k = 0; k < R; ++k) ptr[k + 1] += ptr[k];
    }
    s.sub_cut = cut;
    s.sub_roots = R;
}

// Lanes per node: enough lanes for the widest per-node loop of the level
// (its destinations, a quarter of its descendants), but no more than keeps
// one pass over the level within a 256-thread workgroup.
void default_mapping(HostSym& s)
{
    const int threads = 256;
    int nlev = (int)s.level_ptr.size() - 1;
    s.level_g.assign(std::max(nlev, 1), 1);
    for (int l = 0; l < nlev; ++l) {
        int w = s.level_ptr[l + 1] - s.level_ptr[l];
        int need = 1;
        for (int x = s.level_ptr[l]; x < s.level_ptr[l + 1]; ++x) {
            int p = s.level_nodes[x];
            int ns = s.Lp[p + 1] - s.Lp[p];
            int nr = (s.Rp[p + 1] - s.Rp[p] + 3) / 4;
            need = std::max(need, std::max(ns, nr));
        }
        int g = 1;
        while (g < need && g < 64) g <<= 1;
        int fit = 1;
        while (fit * 2 * w <= threads && fit < 64) fit <<= 1;
        s.level_g[l] = std::max(1, std::min(g, fit));
    }
}

}  // namespace pf
