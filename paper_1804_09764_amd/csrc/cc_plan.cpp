// Template planner (host): rooting, the active/passive partition, table liveness, automorphism
// count, bookkeeping, and the device constant tables (colour-set split lists and fold maps).
//
// Partition (Section 2.1, Figure 1(a); Algorithm 1, "Partition T into subtrees"): the template is
// rooted at rho; the sub-template at a vertex x with children c_1..c_m is built by attaching the
// children's full subtrees one at a time. Attaching c_j is one cut of Eq. 1: active part T' = x
// with c_1..c_{j-1} attached, passive part T'' = the subtree of c_j rooted at c_j. Leaves of the
// partition are single vertices.
#include <algorithm>
#include <cstring>
#include <functional>
#include <map>
#include <numeric>

#include "cc_internal.h"

namespace cc {

int64_t binom(int n, int r) {
    if (r < 0 || n < 0 || r > n) return 0;
    int64_t b = 1;
    for (int i = 1; i <= r; ++i) b = b * (n - r + i) / i;
    return b;
}

int pad_stride(int W) {
    if (W <= 1) return 1;
    if (W <= 16) {
        int s = 1;
        while (s < W) s <<= 1;
        return s;
    }
    return (W + 15) / 16 * 16;
}

namespace {

// colex rank: rank({c_0 < c_1 < ...}) = sum_j C(c_j, j+1), the same over any number of colours.
// Tabulated once for every mask of up to 16 colours: removing the largest element c of a set of
// j elements lowers its rank by C(c, j).
int colex_rank(uint32_t mask) {
    static const std::vector<int> table = [] {
        int B[17][17];
        for (int n = 0; n <= 16; ++n)
            for (int r = 0; r <= 16; ++r) B[n][r] = (int)binom(n, r);
        std::vector<int> t(1u << 16, 0);
        for (uint32_t m = 1; m < (1u << 16); ++m) {
            const int c = 31 - __builtin_clz(m);
            t[m] = t[m ^ (1u << c)] + B[c][__builtin_popcount(m)];
        }
        return t;
    }();
    return table[mask];
}

std::vector<uint32_t> masks_of(int K, int m) {
    std::vector<uint32_t> v;
    for (uint32_t x = 0; x < (1u << K); ++x)
        if (__builtin_popcount(x) == m) v.push_back(x);
    return v;
}

// the low bits of x placed on the set bits of R, lowest first: increasing in x
uint32_t deposit(uint32_t x, uint32_t R) {
    uint32_t out = 0;
    for (uint32_t b = 1; R != 0; R &= R - 1, b <<= 1)
        if (x & b) out |= R & (~R + 1u);
    return out;
}

// the next larger integer with as many set bits as x
uint32_t next_same_popcount(uint32_t x) {
    const uint32_t c = x & (~x + 1u), r = x + c;
    return (((r ^ x) >> 2) / c) | r;
}

// Storage order of the entries of a table row whose sets have m colours out of K: order[pos] =
// colex rank of the set stored at position pos. Rows are read in 128-byte lines of 16 entries,
// and a reader skips the entries whose set holds its own colour, so a line can be skipped only
// when all of its sets share that colour. Lines are therefore filled, as far as possible, with
// 16 sets that share a common subset Q (|Q| = 4, then 3, 2, 1): such a line is skipped for every
// colour of Q. Sets left over keep colex order at the end. Rows of at most 16 entries keep colex
// order.
std::vector<int> table_order(int K, int m) {
    const auto sets = masks_of(K, m);
    const int W = (int)sets.size();
    std::vector<int> order;
    order.reserve((size_t)W);
    if (W <= 16) {
        for (int r = 0; r < W; ++r) order.push_back(r);
        return order;
    }
    std::vector<char> used((size_t)W, 0);
    for (int q = std::min(m, 4); q >= 1; --q)
        for (uint32_t Q : masks_of(K, q)) {
            // the unused supersets of Q in colex order: Q plus the (m-q)-subsets of the other
            // colours, in increasing numeric order
            std::vector<int> cand;
            const uint32_t rest = ((1u << K) - 1u) & ~Q;
            if (m == q) {
                const int r = colex_rank(Q);
                if (!used[(size_t)r]) cand.push_back(r);
            } else {
                for (uint32_t x = (1u << (m - q)) - 1u; x < (1u << (K - q)); x = next_same_popcount(x)) {
                    const int r = colex_rank(Q | deposit(x, rest));
                    if (!used[(size_t)r]) cand.push_back(r);
                }
            }
            const size_t full = cand.size() / 16 * 16;
            for (size_t i = 0; i < full; ++i) {
                order.push_back(cand[i]);
                used[(size_t)cand[i]] = 1;
            }
        }
    // chain the full lines so that neighbouring lines share as many common colours as possible:
    // the lines a reader skips then sit together, and the lines it reads form fewer runs
    const size_t nfull = order.size() / 16;
    std::vector<uint32_t> common(nfull, (1u << K) - 1u);
    for (size_t l = 0; l < nfull; ++l)
        for (size_t i = 0; i < 16; ++i) common[l] &= sets[(size_t)order[l * 16 + i]];
    std::vector<int> chain;
    std::vector<char> taken(nfull, 0);
    for (size_t step = 0; step < nfull; ++step) {
        size_t best = nfull;
        int best_shared = -1;
        for (size_t l = 0; l < nfull; ++l) {
            if (taken[l]) continue;
            const int shared = chain.empty() ? 0 : __builtin_popcount(common[l] & common[(size_t)chain.back()]);
            if (shared > best_shared) {
                best_shared = shared;
                best = l;
            }
        }
        taken[best] = 1;
        chain.push_back((int)best);
    }
    std::vector<int> chained;
    chained.reserve((size_t)W);
    for (int l : chain)
        for (size_t i = 0; i < 16; ++i) chained.push_back(order[(size_t)l * 16 + i]);
    for (int r = 0; r < W; ++r)
        if (!used[(size_t)r]) chained.push_back(r);
    return chained;
}

std::vector<int> inverse(const std::vector<int>& order) {
    std::vector<int> pos(order.size());
    for (size_t i = 0; i < order.size(); ++i) pos[(size_t)order[i]] = (int)i;
    return pos;
}

uint32_t expand_bits(uint32_t m, int c) {  // insert a zero bit at position c
    uint32_t lo = m & ((1u << c) - 1u);
    return lo | ((m >> c) << (c + 1));
}

uint32_t compress_bits(uint32_t m, int c) {  // delete bit position c
    uint32_t lo = m & ((1u << c) - 1u);
    return lo | ((m >> (c + 1)) << c);
}

struct Tree {
    int k;
    std::vector<std::vector<int>> adj;
};

bool load_tree(int k, const int32_t* e, Tree* t, std::string* err) {
    t->k = k;
    t->adj.assign(k, {});
    for (int i = 0; i < k - 1; ++i) {
        int u = e[2 * i], v = e[2 * i + 1];
        if (u < 0 || v < 0 || u >= k || v >= k || u == v) {
            *err = "template edge out of range or a self-loop";
            return false;
        }
        if (std::find(t->adj[u].begin(), t->adj[u].end(), v) != t->adj[u].end()) {
            *err = "duplicate template edge";
            return false;
        }
        t->adj[u].push_back(v);
        t->adj[v].push_back(u);
    }
    std::vector<int> seen(k, 0), st{0};
    seen[0] = 1;
    int cnt = 0;
    while (!st.empty()) {
        int x = st.back();
        st.pop_back();
        ++cnt;
        for (int y : t->adj[x])
            if (!seen[y]) { seen[y] = 1; st.push_back(y); }
    }
    if (cnt != k) {
        *err = "template is not connected (k-1 edges must form a tree)";
        return false;
    }
    return true;
}

std::vector<int> centres(const Tree& t) {
    int k = t.k;
    if (k <= 2) {
        std::vector<int> c;
        for (int i = 0; i < k; ++i) c.push_back(i);
        return c;
    }
    std::vector<int> deg(k), removed(k, 0), layer;
    for (int i = 0; i < k; ++i) {
        deg[i] = (int)t.adj[i].size();
        if (deg[i] == 1) layer.push_back(i);
    }
    int left = k;
    while (left > 2) {
        std::vector<int> nxt;
        for (int x : layer) {
            removed[x] = 1;
            --left;
            for (int y : t.adj[x])
                if (!removed[y] && --deg[y] == 1) nxt.push_back(y);
        }
        layer = nxt;
    }
    std::vector<int> c;
    for (int i = 0; i < k; ++i)
        if (!removed[i]) c.push_back(i);
    return c;
}

// AHU canonical string of the subtree of x (parent p excluded)
std::string canon(const Tree& t, int x, int p) {
    std::vector<std::string> ch;
    for (int y : t.adj[x])
        if (y != p) ch.push_back(canon(t, y, x));
    std::sort(ch.begin(), ch.end());
    std::string s = "(";
    for (auto& c : ch) s += c;
    return s + ")";
}

// automorphisms of the subtree of x that fix x: product over vertices of the factorials of the
// multiplicities of isomorphic child subtrees
double rooted_aut(const Tree& t, int x, int p) {
    double a = 1.0;
    std::map<std::string, int> mult;
    for (int y : t.adj[x])
        if (y != p) {
            a *= rooted_aut(t, y, x);
            mult[canon(t, y, x)]++;
        }
    for (auto& kv : mult)
        for (int i = 2; i <= kv.second; ++i) a *= i;
    return a;
}

// |Aut(T)|: automorphisms fix the centre (or the centre edge as a set)
double tree_aut(const Tree& t) {
    auto c = centres(t);
    if (c.size() == 1) return rooted_aut(t, c[0], -1);
    double a = rooted_aut(t, c[0], c[1]) * rooted_aut(t, c[1], c[0]);
    if (canon(t, c[0], c[1]) == canon(t, c[1], c[0])) a *= 2.0;
    return a;
}

struct Rooted {
    std::vector<int> parent, size;
    std::vector<std::vector<int>> kids;
};

Rooted root_at(const Tree& t, int r) {
    Rooted R;
    R.parent.assign(t.k, -1);
    R.size.assign(t.k, 1);
    R.kids.assign(t.k, {});
    std::function<int(int, int)> dfs = [&](int x, int p) {
        R.parent[x] = p;
        for (int y : t.adj[x])
            if (y != p) {
                R.kids[x].push_back(y);
                R.size[x] += dfs(y, x);
            }
        return R.size[x];
    };
    dfs(r, -1);
    return R;
}

int64_t W_of(int k, int t) { return binom(k - 1, t - 1); }

// combine multiply-adds of attaching children of the given sizes in this order
int64_t chain_combine(int k, const std::vector<int>& sizes) {
    int a = 1;
    int64_t c = 0;
    for (int p : sizes) {
        int s = a + p;
        if (a >= 2) c += W_of(k, s) * binom(s - 1, p);
        a = s;
    }
    return c;
}

// order the children of every vertex: the cheapest combine (exhaustive up to 7 children),
// ties broken towards larger subtrees first; `smallest_first` gives the fixed reference order
void order_children(int k, Rooted* R, bool smallest_first) {
    for (int x = 0; x < k; ++x) {
        auto& ch = R->kids[x];
        std::sort(ch.begin(), ch.end(), [&](int a, int b) {
            if (R->size[a] != R->size[b])
                return smallest_first ? R->size[a] < R->size[b] : R->size[a] > R->size[b];
            return a < b;
        });
        if (smallest_first || ch.size() < 2 || ch.size() > 7) continue;
        std::vector<int> best = ch, perm = ch;
        auto sizes = [&](const std::vector<int>& o) {
            std::vector<int> s;
            for (int y : o) s.push_back(R->size[y]);
            return s;
        };
        int64_t best_c = chain_combine(k, sizes(ch));
        std::sort(perm.begin(), perm.end());
        do {
            int64_t c = chain_combine(k, sizes(perm));
            if (c < best_c) { best_c = c; best = perm; }
        } while (std::next_permutation(perm.begin(), perm.end()));
        ch = best;
    }
}

struct Arena {
    // first-fit allocator over columns
    std::vector<std::pair<int64_t, int64_t>> used;  // (off, len)
    int64_t peak = 0;
    int64_t alloc(int64_t len) {
        std::sort(used.begin(), used.end());
        int64_t off = 0;
        for (auto& u : used) {
            if (u.first - off >= len) break;
            off = std::max(off, u.first + u.second);
        }
        used.push_back({off, len});
        peak = std::max(peak, off + len);
        return off;
    }
    void release(int64_t off) {
        for (size_t i = 0; i < used.size(); ++i)
            if (used[i].first == off) { used.erase(used.begin() + i); return; }
    }
};

struct Schedule {
    std::vector<Split> splits;
    std::vector<Table> tables;
    int64_t arena_cols = 0;
    int64_t live_peak = 0;
};

// AHU canonical string of the rooted subtree of x in R
std::string rcanon(const Rooted& R, int x) {
    std::vector<std::string> ch;
    for (int y : R.kids[x]) ch.push_back(rcanon(R, y));
    std::sort(ch.begin(), ch.end());
    std::string s = "(";
    for (auto& c : ch) s += c;
    return s + ")";
}

Schedule schedule(int k, const Rooted& R, int root) {
    Schedule S;
    Arena A;
    int64_t live = 0;
    std::function<int(int)> compute = [&](int x) -> int {
        int act = -1, a = 1;
        std::vector<std::string> attached;  // canonical forms of the children attached so far
        for (size_t j = 0; j < R.kids[x].size(); ++j) {
            int c = R.kids[x][j];
            int pas = compute(c);
            attached.push_back(rcanon(R, c));
            int p = R.size[c];
            int s = a + p;
            bool last_root = (x == root) && (j + 1 == R.kids[x].size());
            Split sp{};
            sp.s = s; sp.a = a; sp.p = p; sp.act = act; sp.pas = pas;
            sp.Wa = (int)W_of(k, a); sp.Wp = (int)W_of(k, p); sp.Ws = (int)W_of(k, s);
            sp.Nw = (int)binom(k - 1, p);
            sp.npairs = (int)binom(s - 1, p);
            if (last_root) {
                sp.out = -2;
            } else {
                Table t{};
                t.size = s; t.W = sp.Ws; t.stride = pad_stride(t.W);
                std::vector<std::string> sorted_kids = attached;
                std::sort(sorted_kids.begin(), sorted_kids.end());
                t.key = "(";
                for (auto& ck : sorted_kids) t.key += ck;
                t.key += ")";
                t.col_off = A.alloc(t.stride);
                live += t.stride;
                S.tables.push_back(t);
                sp.out = (int)S.tables.size() - 1;
            }
            S.live_peak = std::max(S.live_peak, live);
            if (act >= 0) { A.release(S.tables[act].col_off); live -= S.tables[act].stride; }
            if (pas >= 0) { A.release(S.tables[pas].col_off); live -= S.tables[pas].stride; }
            S.splits.push_back(sp);
            act = sp.out;
            a = s;
        }
        return act;  // -1 when x is a leaf of T
    };
    compute(root);
    S.arena_cols = A.peak;
    return S;
}

// The splits of S that must run when equal rooted sub-templates (equal table keys) are computed
// once: walking from the root split, a table whose key was produced before is reused, and the
// splits that would only feed it are dropped. Tables are renumbered, and the arena is first-fit
// again over the shorter sequence with each table released after its last use.
Schedule share_tables(const Schedule& S) {
    Schedule D;
    if (S.splits.empty()) return D;
    std::vector<int> producer(S.tables.size(), -1);
    for (size_t j = 0; j < S.splits.size(); ++j)
        if (S.splits[j].out >= 0) producer[(size_t)S.splits[j].out] = (int)j;
    std::map<std::string, int> have;
    std::function<int(int)> need = [&](int t) -> int {
        auto it = have.find(S.tables[(size_t)t].key);
        if (it != have.end()) return it->second;
        Split sp = S.splits[(size_t)producer[(size_t)t]];
        sp.act = sp.act >= 0 ? need(sp.act) : -1;
        sp.pas = sp.pas >= 0 ? need(sp.pas) : -1;
        D.tables.push_back(S.tables[(size_t)t]);
        sp.out = (int)D.tables.size() - 1;
        have[S.tables[(size_t)t].key] = sp.out;
        D.splits.push_back(sp);
        return sp.out;
    };
    Split root = S.splits.back();
    root.act = root.act >= 0 ? need(root.act) : -1;
    root.pas = root.pas >= 0 ? need(root.pas) : -1;
    D.splits.push_back(root);
    // liveness over the new sequence
    std::vector<int> last(D.tables.size(), -1);
    for (size_t j = 0; j < D.splits.size(); ++j) {
        if (D.splits[j].act >= 0) last[(size_t)D.splits[j].act] = (int)j;
        if (D.splits[j].pas >= 0) last[(size_t)D.splits[j].pas] = (int)j;
    }
    Arena A;
    int64_t live = 0;
    for (size_t j = 0; j < D.splits.size(); ++j) {
        const Split& sp = D.splits[j];
        if (sp.out >= 0) {
            Table& t = D.tables[(size_t)sp.out];
            t.col_off = A.alloc(t.stride);
            live += t.stride;
        }
        D.live_peak = std::max(D.live_peak, live);
        for (int in : {sp.act, sp.pas == sp.act ? -1 : sp.pas})  // each input once
            if (in >= 0 && last[(size_t)in] == (int)j) {
                A.release(D.tables[(size_t)in].col_off);
                live -= D.tables[(size_t)in].stride;
            }
    }
    D.arena_cols = A.peak;
    return D;
}

}  // namespace

std::vector<int> entry_order(int K, int m) { return table_order(K, m); }

int64_t packed_arena(const cc_plan* P, int B, std::vector<int64_t>* col_off) {
    // the plan's allocation order: each split allocates its output table, then releases the
    // inputs it is the last reader of (a shared table has several readers)
    std::vector<int> last(P->tables.size(), -1);
    for (size_t j = 0; j < P->splits.size(); ++j) {
        if (P->splits[j].act >= 0) last[(size_t)P->splits[j].act] = (int)j;
        if (P->splits[j].pas >= 0) last[(size_t)P->splits[j].pas] = (int)j;
    }
    Arena A;
    col_off->assign(P->tables.size(), 0);
    for (size_t j = 0; j < P->splits.size(); ++j) {
        const Split& sp = P->splits[j];
        if (sp.out >= 0)
            (*col_off)[(size_t)sp.out] = A.alloc(packed_cols(P->tables[(size_t)sp.out].W, B));
        for (int in : {sp.act, sp.pas == sp.act ? -1 : sp.pas})  // each input once
            if (in >= 0 && last[(size_t)in] == (int)j) A.release((*col_off)[(size_t)in]);
    }
    return A.peak;
}

cc_status plan_build(int k, const int32_t* edges, int root, uint32_t flags, cc_plan* P,
                     std::string* err) {
    if (k < 1 || k > kMaxK) {
        *err = "k must be in [1, 16]";
        return CC_ERANGE;
    }
    if (k > 1 && !edges) {
        *err = "edges is NULL";
        return CC_EINVAL;
    }
    Tree t;
    if (!load_tree(k, edges, &t, err)) return CC_EINVAL;
    if (root < -1 || root >= k) {
        *err = "root out of range";
        return CC_EINVAL;
    }
    P->k = k;
    P->edges.assign(edges, edges + 2 * (k - 1));
    P->aut = tree_aut(t);

    // colour-set-edge units on the reference partition (root = centre with the smallest label)
    {
        int c0 = centres(t)[0];
        Rooted R = root_at(t, c0);
        int64_t u = 0;
        for (int x = 0; x < k; ++x)
            if (x != c0) u += (R.size[x] >= 2) ? binom(k, R.size[x]) : 1;
        P->units_per_edge = u;
    }

    const bool reference = (flags & CC_PLAN_CENTRE_SMALLEST) != 0;
    std::vector<int> candidates;
    if (root >= 0) candidates.push_back(root);
    else if (reference) candidates.push_back(centres(t)[0]);
    else for (int r = 0; r < k; ++r) candidates.push_back(r);

    // choose the root: fewest doubles gathered per edge (weighted 256x: one gathered double per
    // edge costs about as much HBM time as 256 combine multiply-adds per vertex at average degree
    // ~30), then the smaller table arena
    const bool share = !reference && (flags & CC_PLAN_NO_SHARING) == 0;
    double best_cost = 1e300;
    Schedule best, best_full;
    Rooted bestR;
    int best_root = candidates[0];
    for (int r : candidates) {
        Rooted R = root_at(t, r);
        order_children(k, &R, reference);
        const Schedule full = schedule(k, R, r);
        const Schedule S = share ? share_tables(full) : full;
        int64_t g = 0, c = 0;
        for (auto& sp : S.splits) {
            if (sp.p >= 2) g += sp.Wp;
            if (sp.a >= 2) c += (int64_t)sp.Ws * sp.npairs;
        }
        double cost = 256.0 * (double)g + (double)c + 1e-6 * (double)S.arena_cols;
        if (cost < best_cost) {
            best_cost = cost;
            best = S;
            best_full = full;
            bestR = R;
            best_root = r;
        }
    }
    P->root = best_root;
    P->splits = best.splits;
    P->tables = best.tables;
    P->arena_cols = best.arena_cols;
    P->peak_live_cols = best.live_peak;

    // bookkeeping (Table 3 counts every split of the partition, shared or not)
    P->t3_memory = P->t3_compute = P->gather_per_edge = P->combine_per_vertex = 0;
    P->max_Nw = 0;
    for (auto& sp : best_full.splits)
        if (sp.out != -2) {
            P->t3_memory += binom(k, sp.s);
            P->t3_compute += binom(k, sp.s) * binom(sp.s, sp.a);
        }
    for (auto& sp : P->splits) {
        if (sp.p >= 2) P->gather_per_edge += sp.Wp;
        if (sp.a >= 2) P->combine_per_vertex += (int64_t)sp.Ws * sp.npairs;
        P->max_Nw = std::max(P->max_Nw, sp.Nw);
    }
    P->max_stride_N = pad_stride(P->max_Nw);

    // device constants
    const int K = k - 1;
    std::vector<uint8_t>& C = P->consts;
    C.clear();
    auto align = [&]() { while (C.size() % 256) C.push_back(0); };
    std::vector<std::vector<int>> orders((size_t)k);  // storage order per set size, built once
    auto order_of = [&](int m) -> const std::vector<int>& {
        if (orders[(size_t)m].empty()) orders[(size_t)m] = table_order(K, m);
        return orders[(size_t)m];
    };
    for (auto& sp : P->splits) {
        sp.split_off = -1;
        sp.fold_off = -1;
        sp.mask_off = -1;
        sp.full_off = -1;
        sp.emap_off = -1;
        sp.Wn = 0;
        sp.Wn_pad = 0;
        sp.lines_need = 0.0;
        sp.proj_src_off = -1;
        sp.proj_fold_off = -1;
        sp.proj_mask_off = -1;
        sp.Cf = (int)binom(k, sp.p);
        // storage orders of the output, active and passive rows (tables of equal size share one)
        const std::vector<int>& order_s = order_of(sp.s - 1);
        const std::vector<int> pos_s = inverse(order_s);
        const std::vector<int> pos_a = inverse(order_of(sp.a - 1));
        const std::vector<int>& order_p = order_of(sp.p - 1);
        if (sp.a >= 2) {
            // for every output set R (|R| = s-1) its p-subsets Q in increasing numeric order:
            // (storage position of R \ Q in the active row, colex rank of Q in N) packed as
            // lo16 | hi16 << 16, layout [j][storage position of R in the output row]
            align();
            sp.split_off = (int64_t)C.size();
            auto outs = masks_of(K, sp.s - 1);
            std::vector<uint32_t> tab((size_t)sp.npairs * outs.size());
            for (size_t r = 0; r < outs.size(); ++r) {
                const uint32_t R = outs[r];
                const uint32_t end = 1u << (sp.s - 1);  // |R| = s - 1
                int j = 0;
                // the p-subsets of R in increasing numeric order: the p-bit patterns over R's bits
                // in increasing order, deposited on them
                for (uint32_t x = (1u << sp.p) - 1u; x < end; x = next_same_popcount(x)) {
                    const uint32_t q = deposit(x, R);
                    const uint32_t ia = (uint32_t)pos_a[(size_t)colex_rank(R & ~q)], in = (uint32_t)colex_rank(q);
                    tab[(size_t)j * outs.size() + (size_t)pos_s[r]] = ia | (in << 16);
                    ++j;
                }
            }
            const uint8_t* b = reinterpret_cast<const uint8_t*>(tab.data());
            C.insert(C.end(), b, b + tab.size() * 4);
        }
        if (sp.p >= 2) {
            // fold map M[cu][cv][j]: passive entry j of a neighbour u (colour cu) is the set
            // R_u (|R_u| = p-1) over the colours other than cu; it adds to N(v, Q) with
            // Q = R_u + {cu} written over the colours other than cv, unless cv is in R_u
            align();
            sp.fold_off = (int64_t)C.size();
            // passive rows in storage order: entry j holds the set of colex rank order_p[j]
            std::vector<uint32_t> rows = masks_of(K, sp.p - 1);
            {
                std::vector<uint32_t> stored(rows.size());
                for (size_t j = 0; j < rows.size(); ++j) stored[j] = rows[(size_t)order_p[j]];
                rows.swap(stored);
            }
            std::vector<uint16_t> tab((size_t)k * k * rows.size(), kNoSlot);
            for (int cu = 0; cu < k; ++cu)
                for (int cv = 0; cv < k; ++cv) {
                    if (cu == cv) continue;
                    for (size_t j = 0; j < rows.size(); ++j) {
                        uint32_t full = expand_bits(rows[j], cu);
                        if (full >> cv & 1u) continue;
                        uint32_t Q = compress_bits(full | (1u << cu), cv);
                        tab[((size_t)cu * k + cv) * rows.size() + j] = (uint16_t)colex_rank(Q);
                    }
                }
            const uint8_t* b = reinterpret_cast<const uint8_t*>(tab.data());
            C.insert(C.end(), b, b + tab.size() * 2);
            // expected 128-byte lines of a stored row holding an entry a centre needs (the
            // centre's colour is uniform over the k-1 colours of the row)
            {
                const size_t W = rows.size();
                int64_t lines = 0;
                for (int x = 0; x < K; ++x)
                    for (size_t l = 0; l < W; l += 16) {
                        bool any = false;
                        for (size_t j = l; j < std::min(W, l + 16); ++j) any = any || !((rows[j] >> x) & 1u);
                        lines += any ? 1 : 0;
                    }
                sp.lines_need = K > 0 ? (double)lines / K : 0.0;
            }
            if (sp.Wp > 64) {
                // projected rows: for (cu, cv) the storage positions j whose fold target is a slot,
                // ordered by that slot (the colex rank of the set over the colours other than cv),
                // and the slots themselves; Wn = C(k-2, p-1) of them for cu != cv
                sp.Wn = (int)binom(k - 2, sp.p - 1);
                sp.Wn_pad = pad_stride(sp.Wn);
                const size_t W = rows.size(), Wn = (size_t)sp.Wn;
                std::vector<uint16_t> src((size_t)k * k * Wn, 0), dst((size_t)k * k * Wn, kNoSlot);
                for (int cu = 0; cu < k; ++cu)
                    for (int cv = 0; cv < k; ++cv) {
                        if (cu == cv) continue;
                        const uint16_t* f = &tab[((size_t)cu * k + cv) * W];
                        std::vector<std::pair<uint16_t, uint16_t>> need;
                        for (size_t j = 0; j < W; ++j)
                            if (f[j] != kNoSlot) need.push_back({f[j], (uint16_t)j});
                        std::sort(need.begin(), need.end());
                        if (need.size() != Wn) {
                            *err = "internal: projected row width";
                            return CC_EINTERNAL;
                        }
                        for (size_t q = 0; q < Wn; ++q) {
                            src[((size_t)cu * k + cv) * Wn + q] = need[q].second;
                            dst[((size_t)cu * k + cv) * Wn + q] = need[q].first;
                        }
                    }
                align();
                sp.proj_src_off = (int64_t)C.size();
                const uint8_t* bs = reinterpret_cast<const uint8_t*>(src.data());
                C.insert(C.end(), bs, bs + src.size() * 2);
                align();
                sp.proj_fold_off = (int64_t)C.size();
                const uint8_t* bd = reinterpret_cast<const uint8_t*>(dst.data());
                C.insert(C.end(), bd, bd + dst.size() * 2);
                align();
                sp.proj_mask_off = (int64_t)C.size();
                C.insert(C.end(), Wn * 2, 0);
            }
            // set of passive entry j as a bit mask over the k-1 colours other than the
            // neighbour's: entry j is of no use to v when it contains col(v)'s position there
            align();
            sp.mask_off = (int64_t)C.size();
            std::vector<uint16_t> mk(rows.size());
            for (size_t j = 0; j < rows.size(); ++j) mk[j] = (uint16_t)rows[j];
            const uint8_t* bm = reinterpret_cast<const uint8_t*>(mk.data());
            C.insert(C.end(), bm, bm + mk.size() * 2);
            // packed layout: FM[cu][j] = colex rank over all k colours of R_u + {cu}
            align();
            sp.full_off = (int64_t)C.size();
            std::vector<uint16_t> fm((size_t)k * rows.size(), kNoSlot);
            for (int cu = 0; cu < k; ++cu)
                for (size_t j = 0; j < rows.size(); ++j)
                    fm[(size_t)cu * rows.size() + j] = (uint16_t)colex_rank(expand_bits(rows[j], cu) | (1u << cu));
            const uint8_t* bf = reinterpret_cast<const uint8_t*>(fm.data());
            C.insert(C.end(), bf, bf + fm.size() * 2);
        }
        // packed layout: E[cv][q] = colex rank over all k colours of the p-set whose rank over the
        // colours other than cv is q. With a = 1 the combine reads it by output position (the
        // output set is that p-set plus cv), so q runs over the output row's storage order.
        {
            align();
            sp.emap_off = (int64_t)C.size();
            auto qs = masks_of(K, sp.p);
            std::vector<uint16_t> em((size_t)k * qs.size());
            for (int cv = 0; cv < k; ++cv)
                for (size_t q = 0; q < qs.size(); ++q) {
                    const size_t qq = sp.a == 1 ? (size_t)order_s[q] : q;
                    em[(size_t)cv * qs.size() + q] = (uint16_t)colex_rank(expand_bits(qs[qq], cv));
                }
            const uint8_t* be = reinterpret_cast<const uint8_t*>(em.data());
            C.insert(C.end(), be, be + em.size() * 2);
        }
        // a = 1: the split list is the entry of N (colex rank) stored at each output position
        if (sp.a == 1) {
            align();
            sp.split_off = (int64_t)C.size();
            std::vector<uint32_t> om((size_t)sp.Ws);
            for (int r = 0; r < sp.Ws; ++r) om[(size_t)r] = (uint32_t)order_s[(size_t)r];
            const uint8_t* bo = reinterpret_cast<const uint8_t*>(om.data());
            C.insert(C.end(), bo, bo + om.size() * 4);
        }
    }
    align();
    if (C.empty()) C.resize(256, 0);
    return CC_OK;
}

}  // namespace cc
