// Host symbolic analysis: condensed pattern, ordering, elimination tree,
// column counts, supernodes, multifrontal maps and the level schedule.
//
// Pattern (Sec. 2.2 K1, Sec. 3.1 eq:kkt:hykkt, Sec. 3.2 eq:liftedkkt):
//   pattern(K) = pattern(W) U diag U { (i, j) : J_ri != 0 and J_rj != 0 }
// with J = [G; H]; K_gamma adds gamma G^T G, whose pattern is already in
// J^T J, so one analysis serves both formulations.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdint>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "analysis.hpp"

namespace ckkt {

namespace {

std::string check_csr(const char* name, int64_t nrows, int64_t ncols, const std::vector<int32_t>& ptr,
                      const std::vector<int32_t>& idx, bool lower) {
    if ((int64_t)ptr.size() != nrows + 1) return std::string(name) + ": ptr has wrong length";
    if (ptr[0] != 0) return std::string(name) + ": ptr[0] != 0";
    for (int64_t i = 0; i < nrows; ++i) {
        if (ptr[i + 1] < ptr[i]) return std::string(name) + ": ptr decreases";
    }
    if ((int64_t)idx.size() != (int64_t)ptr[nrows]) return std::string(name) + ": idx has wrong length";
    for (int64_t i = 0; i < nrows; ++i) {
        for (int32_t k = ptr[i]; k < ptr[i + 1]; ++k) {
            int32_t c = idx[k];
            if (c < 0 || c >= ncols) return std::string(name) + ": column out of range";
            if (lower && c > i) return std::string(name) + ": entry above the diagonal";
            if (k > ptr[i] && idx[k - 1] >= c) return std::string(name) + ": columns not strictly increasing";
        }
    }
    return "";
}

}  // namespace

std::string validate(const PatternIn& p) {
    if (p.n < 0 || p.m_eq < 0 || p.m_ineq < 0) return "negative dimension";
    if (p.n > (int64_t)1 << 30 || p.m_eq + p.m_ineq > (int64_t)1 << 30) return "dimension too large";
    std::string e = check_csr("W", p.n, p.n, p.w_ptr, p.w_idx, true);
    if (!e.empty()) return e;
    e = check_csr("G", p.m_eq, p.n, p.g_ptr, p.g_idx, false);
    if (!e.empty()) return e;
    e = check_csr("H", p.m_ineq, p.n, p.h_ptr, p.h_idx, false);
    return e;
}

namespace {

// Off-diagonal pairs (i > j) of W + J^T J over the variables [v0, v1), the
// equality rows [g0, g1) and the inequality rows [h0, h1), sorted and
// unique; rows of J flagged in `dense` contribute nothing.
std::vector<uint64_t> pattern_keys_range(const PatternIn& p, const std::vector<char>& dense, int32_t v0, int32_t v1,
                                         int32_t g0, int32_t g1, int32_t h0, int32_t h1) {
    const int32_t me = (int32_t)p.m_eq;
    auto row = [&](int32_t r, const int32_t*& b, const int32_t*& e) {
        if (r < me) { b = p.g_idx.data() + p.g_ptr[r]; e = p.g_idx.data() + p.g_ptr[r + 1]; }
        else { b = p.h_idx.data() + p.h_ptr[r - me]; e = p.h_idx.data() + p.h_ptr[r - me + 1]; }
    };
    auto rows = [&](auto&& fn) {
        for (int32_t r = g0; r < g1; ++r) fn(r);
        for (int32_t r = me + h0; r < me + h1; ++r) fn(r);
    };
    std::vector<uint64_t> keys;
    {
        int64_t est = (int64_t)p.w_ptr[v1] - p.w_ptr[v0];
        rows([&](int32_t r) {
            const int32_t *b, *e;
            row(r, b, e);
            const int64_t q = dense[r] ? 0 : e - b;
            est += q * (q - 1) / 2;
        });
        keys.reserve(est);
    }
    for (int32_t i = v0; i < v1; ++i)
        for (int32_t k = p.w_ptr[i]; k < p.w_ptr[i + 1]; ++k)
            if (p.w_idx[k] != i) keys.push_back(((uint64_t)i << 32) | (uint32_t)p.w_idx[k]);
    rows([&](int32_t r) {
        if (dense[r]) return;
        const int32_t *b, *e;
        row(r, b, e);
        for (const int32_t* a = b; a < e; ++a)
            for (const int32_t* c = a + 1; c < e; ++c)
                keys.push_back(((uint64_t)*c << 32) | (uint32_t)*a);  // cols increasing: *c > *a
    });
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    return keys;
}

std::vector<uint64_t> pattern_keys(const PatternIn& p, const std::vector<char>& dense) {
    return pattern_keys_range(p, dense, 0, (int32_t)p.n, 0, (int32_t)p.m_eq, 0, (int32_t)p.m_ineq);
}

// The same for a block-diagonal pattern, block by block on up to `threads`
// host threads: the blocks' variable ranges increase, so their sorted key
// lists concatenate into the sorted list of the whole.
std::vector<uint64_t> block_pattern_keys(const PatternIn& p, const std::vector<char>& dense, const AnalyzeOptions& o) {
    const std::vector<int32_t>& bn = *o.block_n;
    const std::vector<int32_t>& bg = *o.block_meq;
    const std::vector<int32_t>& bh = *o.block_mineq;
    const int nb = (int)bn.size() - 1;
    std::vector<std::vector<uint64_t>> part(nb);
    std::atomic<int> next{0};
    auto work = [&]() {
        for (int i; (i = next.fetch_add(1)) < nb;)
            part[i] = pattern_keys_range(p, dense, bn[i], bn[i + 1], bg[i], bg[i + 1], bh[i], bh[i + 1]);
    };
    run_threads(std::max(1, std::min(o.threads, nb)), [&](int) { work(); });
    size_t total = 0;
    for (auto& v : part) total += v.size();
    std::vector<uint64_t> keys;
    keys.reserve(total);
    for (auto& v : part) {
        keys.insert(keys.end(), v.begin(), v.end());
        std::vector<uint64_t>().swap(v);
    }
    return keys;
}

Graph graph_of(int32_t n, const std::vector<uint64_t>& keys) {
    Graph g;
    g.n = n;
    g.ptr.assign(n + 1, 0);
    for (uint64_t k : keys) {
        g.ptr[(k >> 32) + 1]++;
        g.ptr[(uint32_t)k + 1]++;
    }
    for (int32_t i = 0; i < n; ++i) g.ptr[i + 1] += g.ptr[i];
    g.adj.resize(g.ptr[n]);
    std::vector<int32_t> fill(g.ptr.begin(), g.ptr.end() - 1);
    for (uint64_t k : keys) {
        int32_t i = (int32_t)(k >> 32), j = (int32_t)(uint32_t)k;
        g.adj[fill[i]++] = j;
        g.adj[fill[j]++] = i;
    }
    return g;
}

std::vector<char> dense_mask(const PatternIn& p, int dense_row_min) {
    const int32_t me = (int32_t)p.m_eq, mi = (int32_t)p.m_ineq;
    std::vector<char> dense(me + mi, 0);
    if (dense_row_min > 0) {
        for (int32_t r = 0; r < me; ++r) dense[r] = p.g_ptr[r + 1] - p.g_ptr[r] >= dense_row_min;
        for (int32_t r = 0; r < mi; ++r) dense[me + r] = p.h_ptr[r + 1] - p.h_ptr[r] >= dense_row_min;
    }
    return dense;
}

}  // namespace

std::vector<int32_t> order_pattern(const PatternIn& p, int dense_row_min) {
    const int32_t n = (int32_t)p.n;
    if (n <= 1) {
        std::vector<int32_t> id(n);
        std::iota(id.begin(), id.end(), 0);
        return id;
    }
    return amd_order(graph_of(n, pattern_keys(p, dense_mask(p, dense_row_min))));
}

namespace {

// Elimination tree of the ordered pattern, its postorder (children in
// increasing order), the K lower CSC in the postordered numbering and the
// column counts of L, diagonal included.
std::string order_host(int32_t n, const std::vector<uint64_t>& keys, const std::vector<int32_t>& perm0,
                       const std::vector<int32_t>& ip0, Plan& P, std::vector<int32_t>& parent,
                       std::vector<int64_t>& cnt) {
    // ---- elimination tree of the permuted matrix (Liu, with path compression)
    auto etree_of = [&](const std::vector<int32_t>& ip, std::vector<int32_t>& parent) {
        // lower-row lists in the new numbering: for row I, columns J < I
        std::vector<int32_t> rp(n + 1, 0);
        for (uint64_t k : keys) {
            int32_t I = ip[(int32_t)(k >> 32)], J = ip[(int32_t)(uint32_t)k];
            rp[std::max(I, J) + 1]++;
        }
        for (int32_t i = 0; i < n; ++i) rp[i + 1] += rp[i];
        std::vector<int32_t> rc(rp[n]);
        {
            std::vector<int32_t> fill(rp.begin(), rp.end() - 1);
            for (uint64_t k : keys) {
                int32_t I = ip[(int32_t)(k >> 32)], J = ip[(int32_t)(uint32_t)k];
                rc[fill[std::max(I, J)]++] = std::min(I, J);
            }
        }
        parent.assign(n, -1);
        std::vector<int32_t> anc(n, -1);
        for (int32_t i = 0; i < n; ++i) {
            for (int32_t t = rp[i]; t < rp[i + 1]; ++t) {
                int32_t j = rc[t];
                while (j != -1 && j < i) {
                    int32_t nx = anc[j];
                    anc[j] = i;
                    if (nx == -1) { parent[j] = i; break; }
                    j = nx;
                }
            }
        }
        return std::make_pair(std::move(rp), std::move(rc));
    };
    std::vector<int32_t> par0;
    etree_of(ip0, par0);

    // ---- postorder (children in increasing order), then relabel
    std::vector<int32_t> post;
    post.reserve(n);
    {
        std::vector<int32_t> chead(n, -1), cnext(n, -1);
        for (int32_t j = n - 1; j >= 0; --j)
            if (par0[j] >= 0) { cnext[j] = chead[par0[j]]; chead[par0[j]] = j; }
        std::vector<int32_t> stack;
        for (int32_t r = 0; r < n; ++r) {
            if (par0[r] != -1) continue;
            stack.push_back(r);
            while (!stack.empty()) {
                int32_t v = stack.back();
                if (chead[v] >= 0) {
                    int32_t c = chead[v];
                    chead[v] = cnext[c];
                    stack.push_back(c);
                } else {
                    stack.pop_back();
                    post.push_back(v);
                }
            }
        }
    }
    if ((int32_t)post.size() != n) return "internal: postorder incomplete";
    P.perm.resize(n);
    P.iperm.resize(n);
    for (int32_t k = 0; k < n; ++k) P.perm[k] = perm0[post[k]];
    for (int32_t k = 0; k < n; ++k) P.iperm[P.perm[k]] = k;

    auto rows = etree_of(P.iperm, parent);
    const std::vector<int32_t>& rp = rows.first;   // lower rows: row i -> columns j < i
    const std::vector<int32_t>& rc = rows.second;
    for (int32_t j = 0; j < n; ++j)
        if (parent[j] != -1 && parent[j] <= j) return "internal: etree not postordered";

    // ---- K lower CSC (new numbering), rows sorted, diagonal first
    P.kcolptr.assign(n + 1, 0);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t t = rp[i]; t < rp[i + 1]; ++t) P.kcolptr[rc[t] + 1]++;
    for (int32_t j = 0; j < n; ++j) P.kcolptr[j + 1] += P.kcolptr[j] + 1;  // +1 diagonal
    const int64_t nnzk = P.kcolptr[n];
    P.krow.resize(nnzk);
    {
        std::vector<int32_t> fill(n);
        for (int32_t j = 0; j < n; ++j) { P.krow[P.kcolptr[j]] = j; fill[j] = P.kcolptr[j] + 1; }
        for (int32_t i = 0; i < n; ++i)  // rows in increasing order -> sorted columns
            for (int32_t t = rp[i]; t < rp[i + 1]; ++t) P.krow[fill[rc[t]]++] = i;
    }

    // ---- column counts via row subtrees: L(i, j) != 0 iff j on the path from
    //      some k in row i of K (k < i) up to i in the etree
    cnt.assign(n, 1);
    {
        std::vector<int32_t> mk(n, -1);
        for (int32_t i = 0; i < n; ++i) {
            mk[i] = i;
            for (int32_t t = rp[i]; t < rp[i + 1]; ++t) {
                int32_t j = rc[t];
                while (mk[j] != i) {
                    mk[j] = i;
                    cnt[j]++;
                    j = parent[j];
                    if (j < 0) return "internal: row subtree escaped the etree";
                }
            }
        }
    }
    return "";
}

// Row lists of the fronts (own columns, then the rows below in increasing
// order; children before parents), the position of every child row inside
// its parent front and of every K entry inside its own front.  sn_rowptr is
// set from the column counts beforehand.
std::string fronts_host(Plan& P, const std::vector<int64_t>& cnt, const std::vector<int32_t>& col2sn) {
    const int32_t n = P.n, ns = P.ns;
    const int64_t nnzk = P.kcolptr[n];
    // ---- front row structures (children before parents)
    std::vector<std::vector<int32_t>> R(ns);
    {
        std::vector<int32_t> stamp(n, -1);
        for (int32_t s = 0; s < ns; ++s) {
            int32_t c0 = P.sn_start[s], c1 = P.sn_start[s + 1];
            auto& Rs = R[s];
            for (int32_t j = c0; j < c1; ++j)
                for (int32_t t = P.kcolptr[j]; t < P.kcolptr[j + 1]; ++t) {
                    int32_t i = P.krow[t];
                    if (i >= c1 && stamp[i] != s) { stamp[i] = s; Rs.push_back(i); }
                }
            for (int32_t q = P.child_ptr[s]; q < P.child_ptr[s + 1]; ++q)
                for (int32_t i : R[P.child_list[q]])
                    if (i >= c1 && stamp[i] != s) { stamp[i] = s; Rs.push_back(i); }
            std::sort(Rs.begin(), Rs.end());
            if ((int64_t)Rs.size() != cnt[c1 - 1] - 1) return "internal: supernode structure mismatch";
        }
    }
    P.sn_rows.resize(P.sn_rowptr[ns]);
    for (int32_t s = 0; s < ns; ++s) {
        int32_t c0 = P.sn_start[s], c1 = P.sn_start[s + 1];
        int32_t o0 = P.sn_rowptr[s];
        for (int32_t j = c0; j < c1; ++j) P.sn_rows[o0 + j - c0] = j;
        std::copy(R[s].begin(), R[s].end(), P.sn_rows.begin() + o0 + (c1 - c0));
    }
    auto pos_in = [&](int32_t s, int32_t i) -> int32_t {
        int32_t c0 = P.sn_start[s], c1 = P.sn_start[s + 1];
        if (i >= c0 && i < c1) return i - c0;
        auto it = std::lower_bound(R[s].begin(), R[s].end(), i);
        if (it == R[s].end() || *it != i) return -1;
        return (c1 - c0) + (int32_t)(it - R[s].begin());
    };
    P.relmap.assign(P.sn_rows.size(), -1);
    for (int32_t s = 0; s < ns; ++s) {
        int32_t ps = P.sn_parent[s];
        if (ps < 0) continue;
        int32_t w = P.sn_start[s + 1] - P.sn_start[s];
        for (size_t a = 0; a < R[s].size(); ++a) {
            int32_t q = pos_in(ps, R[s][a]);
            if (q < 0) return "internal: child row missing from parent front";
            P.relmap[P.sn_rowptr[s] + w + a] = q;
        }
    }
    P.kmap.resize(nnzk);
    for (int32_t j = 0; j < n; ++j) {
        int32_t s = col2sn[j];
        for (int32_t t = P.kcolptr[j]; t < P.kcolptr[j + 1]; ++t) {
            int32_t q = pos_in(s, P.krow[t]);
            if (q < 0) return "internal: K entry outside its front";
            P.kmap[t] = q;
        }
    }
    return "";
}

// K slot of every product J_ra J_rb (a <= b) of the kept rows, grouped by
// slot with the products in row order inside a slot.
std::string products_host(Plan& P, const std::vector<char>& dense, int threads) {
    const int32_t n = P.n, m = P.m;
    const int64_t nnzk = P.kcolptr[n];
    auto slot_of = [&](int32_t I, int32_t J) -> int32_t {  // I >= J, new numbering
        auto b = P.krow.begin() + P.kcolptr[J], e = P.krow.begin() + P.kcolptr[J + 1];
        auto it = std::lower_bound(b, e, I);
        if (it == e || *it != I) return -1;
        return (int32_t)(it - P.krow.begin());
    };
    {
        // products (a <= b) of every kept row, numbered row by row; their K
        // slots are looked up on host threads, then a counting sort by slot
        // keeps rows increasing inside a slot
        std::vector<int64_t> poff(m + 1, 0);
        for (int32_t r = 0; r < m; ++r) {
            const int64_t q = dense[r] ? 0 : P.j_ptr[r + 1] - P.j_ptr[r];
            poff[r + 1] = poff[r] + q * (q + 1) / 2;
        }
        std::vector<int32_t> pslot(poff[m]);
        std::atomic<bool> missing{false};
        auto lookup = [&](int32_t r0, int32_t r1) {
            for (int32_t r = r0; r < r1; ++r) {
                if (dense[r]) continue;
                int64_t k = poff[r];
                for (int32_t a = P.j_ptr[r]; a < P.j_ptr[r + 1]; ++a)
                    for (int32_t b = a; b < P.j_ptr[r + 1]; ++b) {
                        const int32_t I = P.iperm[P.j_col[a]], J = P.iperm[P.j_col[b]];
                        const int32_t sl = slot_of(std::max(I, J), std::min(I, J));
                        if (sl < 0) missing = true;
                        pslot[k++] = sl;
                    }
            }
        };
        const int nth = std::max(1, std::min(threads, m / 65536 + 1));
        run_threads(nth, [&](int t) {
            lookup((int32_t)((int64_t)m * t / nth), (int32_t)((int64_t)m * (t + 1) / nth));
        });
        if (missing) return "internal: J product missing from K";
        P.prod_ptr.assign(nnzk + 1, 0);
        for (int32_t sl : pslot) P.prod_ptr[sl + 1]++;
        for (int64_t t = 0; t < nnzk; ++t) P.prod_ptr[t + 1] += P.prod_ptr[t];
        P.prod_r.resize(pslot.size());
        P.prod_a.resize(pslot.size());
        P.prod_b.resize(pslot.size());
        std::vector<int32_t> fill(P.prod_ptr.begin(), P.prod_ptr.end() - 1);
        int64_t k = 0;
        for (int32_t r = 0; r < m; ++r) {
            if (dense[r]) continue;
            for (int32_t a = P.j_ptr[r]; a < P.j_ptr[r + 1]; ++a)
                for (int32_t b = a; b < P.j_ptr[r + 1]; ++b) {
                    const int32_t at = fill[pslot[k++]]++;
                    P.prod_r[at] = r;
                    P.prod_a[at] = a;
                    P.prod_b[at] = b;
                }
        }
    }
    return "";
}

}  // namespace

std::string analyze(const PatternIn& p, const AnalyzeOptions& o, Plan& P) {
    auto t0 = std::chrono::steady_clock::now();
    std::string err = validate(p);
    if (!err.empty()) return err;
    const int32_t n = (int32_t)p.n;
    P.n = n;
    P.m_eq = (int32_t)p.m_eq;
    P.m_ineq = (int32_t)p.m_ineq;
    P.m = P.m_eq + P.m_ineq;
    P.nnz_w = (int64_t)p.w_idx.size();
    P.nnz_g = (int64_t)p.g_idx.size();
    P.nnz_h = (int64_t)p.h_idx.size();
    const int32_t m = P.m;

    // ---- J = [G; H]; the value index of an entry equals its position
    P.j_ptr.assign(m + 1, 0);
    for (int32_t r = 0; r < P.m_eq; ++r) P.j_ptr[r + 1] = p.g_ptr[r + 1];
    for (int32_t r = 0; r < P.m_ineq; ++r) P.j_ptr[P.m_eq + r + 1] = (int32_t)P.nnz_g + p.h_ptr[r + 1];
    P.j_col.resize(P.nnz_g + P.nnz_h);
    std::copy(p.g_idx.begin(), p.g_idx.end(), P.j_col.begin());
    std::copy(p.h_idx.begin(), p.h_idx.end(), P.j_col.begin() + P.nnz_g);

    // ---- dense rows: kept out of K (their J^T J block would fill it)
    const std::vector<char> dense = dense_mask(p, o.dense_row_min);
    P.dense_rows.clear();
    for (int32_t r = 0; r < m; ++r)
        if (dense[r]) P.dense_rows.push_back(r);

    // ---- unique off-diagonal pairs (i > j) of W + J^T J, original numbering,
    // and the symmetric graph for the ordering
    const bool blocks = o.block_n && o.block_meq && o.block_mineq && o.block_n->size() > 1 &&
                        o.block_meq->size() == o.block_n->size() && o.block_mineq->size() == o.block_n->size() &&
                        o.block_n->back() == n && o.block_meq->back() == P.m_eq && o.block_mineq->back() == P.m_ineq;
    const std::vector<uint64_t> keys = blocks ? block_pattern_keys(p, dense, o) : pattern_keys(p, dense);
    std::vector<int32_t> perm0;
    if (o.ordering == 1 || n <= 1) {
        perm0.resize(n);
        std::iota(perm0.begin(), perm0.end(), 0);
    } else if (o.perm) {
        perm0 = *o.perm;  // checked below like any ordering
    } else {
        perm0 = amd_order(graph_of(n, keys));
    }
    if ((int32_t)perm0.size() != n) return "internal: ordering is not a permutation";
    std::vector<int32_t> ip0(n, -1);
    for (int32_t k = 0; k < n; ++k) {
        if (perm0[k] < 0 || perm0[k] >= n || ip0[perm0[k]] >= 0) return "internal: ordering is not a permutation";
        ip0[perm0[k]] = k;
    }

    auto since = [](std::chrono::steady_clock::time_point a) {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - a).count();
    };
    P.order_seconds = since(t0);
    P.symbolic_seconds = 0.0;
    std::vector<int32_t> parent;
    std::vector<int64_t> cnt;
    auto ts = std::chrono::steady_clock::now();
    err = o.device ? o.device->order(n, keys, perm0, ip0, P, parent, cnt)
                   : order_host(n, keys, perm0, ip0, P, parent, cnt);
    P.symbolic_seconds += since(ts);
    if (!err.empty()) return err;
    const int64_t nnzk = P.kcolptr[n];
    P.nnz_l = 0;
    P.flops = 0.0;
    for (int32_t j = 0; j < n; ++j) {
        P.nnz_l += cnt[j];
        double eta = (double)(cnt[j] - 1);
        P.flops += eta * eta + 2.0 * eta + 1.0;
    }
    // ---- fundamental supernodes
    std::vector<int32_t> nchild(n, 0);
    for (int32_t j = 0; j < n; ++j)
        if (parent[j] >= 0) nchild[parent[j]]++;
    std::vector<int32_t> fs_first;
    for (int32_t j = 0; j < n; ++j) {
        bool cont = j > 0 && parent[j - 1] == j && cnt[j - 1] == cnt[j] + 1 && nchild[j] == 1;
        if (!cont) fs_first.push_back(j);
    }
    const int32_t ns0 = (int32_t)fs_first.size();
    fs_first.push_back(n);
    std::vector<int32_t> col2fs(n);
    for (int32_t s = 0; s < ns0; ++s)
        for (int32_t j = fs_first[s]; j < fs_first[s + 1]; ++j) col2fs[j] = s;

    // ---- relaxed amalgamation, top-down along chains of last children
    std::vector<int32_t> grp(ns0);
    std::vector<int32_t> g_first(ns0), g_w(ns0);
    std::vector<int64_t> g_r(ns0), g_true(ns0);
    for (int32_t s = ns0 - 1; s >= 0; --s) {
        int32_t c0 = fs_first[s], c1 = fs_first[s + 1];
        int32_t w = c1 - c0;
        int64_t r = cnt[c1 - 1] - 1;
        int64_t tr = 0;
        for (int32_t j = c0; j < c1; ++j) tr += cnt[j];
        int32_t pj = parent[c1 - 1];
        grp[s] = s;
        g_first[s] = c0; g_w[s] = w; g_r[s] = r; g_true[s] = tr;
        if (!o.relax || pj < 0) continue;
        int32_t gp = grp[col2fs[pj]];
        if (g_first[gp] != c1) continue;  // not adjacent (not the last child)
        int64_t wn = (int64_t)w + g_w[gp];
        int64_t f = wn + g_r[gp];
        int64_t stored = wn * f - wn * (wn - 1) / 2;
        int64_t truen = tr + g_true[gp];
        double zf = (double)(stored - truen) / (double)stored;
        bool merge = wn <= 4 || (wn <= 16 && zf < 0.5) || (wn <= 48 && zf < 0.15) || zf < 0.05;
        if (merge) {
            grp[s] = gp;
            g_first[gp] = c0;
            g_w[gp] = (int32_t)wn;
            g_true[gp] = truen;
        }
    }
    // final supernodes in increasing column order
    P.sn_start.clear();
    for (int32_t s = 0; s < ns0; ++s)
        if (grp[s] == s) P.sn_start.push_back(g_first[s]);
    std::sort(P.sn_start.begin(), P.sn_start.end());
    const int32_t ns = (int32_t)P.sn_start.size();
    P.ns = ns;
    P.sn_start.push_back(n);
    std::vector<int32_t> col2sn(n);
    for (int32_t s = 0; s < ns; ++s)
        for (int32_t j = P.sn_start[s]; j < P.sn_start[s + 1]; ++j) col2sn[j] = s;
    P.sn_parent.assign(ns, -1);
    for (int32_t s = 0; s < ns; ++s) {
        int32_t pj = parent[P.sn_start[s + 1] - 1];
        if (pj >= 0) {
            P.sn_parent[s] = col2sn[pj];
            if (P.sn_parent[s] <= s) return "internal: supernode tree not ordered";
        }
    }
    P.child_ptr.assign(ns + 1, 0);
    for (int32_t s = 0; s < ns; ++s)
        if (P.sn_parent[s] >= 0) P.child_ptr[P.sn_parent[s] + 1]++;
    for (int32_t s = 0; s < ns; ++s) P.child_ptr[s + 1] += P.child_ptr[s];
    P.child_list.resize(P.child_ptr[ns]);
    {
        std::vector<int32_t> fill(P.child_ptr.begin(), P.child_ptr.end() - 1);
        for (int32_t s = 0; s < ns; ++s)
            if (P.sn_parent[s] >= 0) P.child_list[fill[P.sn_parent[s]]++] = s;
    }

    // ---- front row structures: sizes from the column counts
    P.sn_rowptr.assign(ns + 1, 0);
    for (int32_t s = 0; s < ns; ++s) {
        const int32_t c0 = P.sn_start[s], c1 = P.sn_start[s + 1];
        P.sn_rowptr[s + 1] = P.sn_rowptr[s] + (c1 - c0) + (int32_t)(cnt[c1 - 1] - 1);
    }
    ts = std::chrono::steady_clock::now();
    err = o.device ? o.device->fronts(P) : fronts_host(P, cnt, col2sn);
    P.symbolic_seconds += since(ts);
    if (!err.empty()) return err;
    P.kcol.resize(nnzk);
    for (int32_t j = 0; j < n; ++j)
        for (int32_t t = P.kcolptr[j]; t < P.kcolptr[j + 1]; ++t) P.kcol[t] = j;

    // ---- factor arena layout
    P.l_off.resize(ns);
    P.u_off.resize(ns);
    P.u_ld.resize(ns);
    P.big.assign(ns, 0);
    P.arena = 0;
    P.nnz_l_stored = 0;
    P.max_front = 0;
    P.n_big = 0;
    for (int32_t s = 0; s < ns; ++s) {
        int64_t w = P.sn_start[s + 1] - P.sn_start[s];
        int64_t f = P.sn_rowptr[s + 1] - P.sn_rowptr[s];
        int64_t r = f - w;
        P.max_front = std::max<int32_t>(P.max_front, (int32_t)f);
        P.nnz_l_stored += w * f - w * (w - 1) / 2;
        bool big = f > o.big_front;
        P.big[s] = big ? 1 : 0;
        P.n_big += big ? 1 : 0;
        int64_t start = (P.arena + 7) & ~(int64_t)7;
        P.l_off[s] = start;
        if (big) {
            P.u_off[s] = start + w + w * f;
            P.u_ld[s] = (int32_t)f;
            P.arena = start + f * f;
        } else {
            P.u_off[s] = start + f * w;
            P.u_ld[s] = (int32_t)std::max<int64_t>(r, 1);
            P.arena = start + f * w + r * r;
        }
    }
    P.arena = (P.arena + 7) & ~(int64_t)7;

    // ---- children contributions by destination front position
    {
        const size_t nrows = P.sn_rows.size();
        P.cb_ptr.assign(nrows + 1, 0);
        for (int32_t c = 0; c < ns; ++c) {
            int32_t p = P.sn_parent[c];
            if (p < 0) continue;
            int32_t wc = P.sn_start[c + 1] - P.sn_start[c];
            int32_t rc = P.sn_rowptr[c + 1] - P.sn_rowptr[c] - wc;
            for (int32_t a = 0; a < rc; ++a) P.cb_ptr[P.sn_rowptr[p] + P.relmap[P.sn_rowptr[c] + wc + a] + 1]++;
        }
        for (size_t q = 0; q < nrows; ++q) P.cb_ptr[q + 1] += P.cb_ptr[q];
        P.cb_src.resize(P.cb_ptr[nrows]);
        P.cb_len.resize(P.cb_ptr[nrows]);
        P.cb_uoff.resize(P.cb_ptr[nrows]);
        std::vector<int32_t> fill(P.cb_ptr.begin(), P.cb_ptr.end() - 1);
        for (int32_t p = 0; p < ns; ++p)
            for (int32_t t = P.child_ptr[p]; t < P.child_ptr[p + 1]; ++t) {  // child order
                int32_t c = P.child_list[t];
                int32_t wc = P.sn_start[c + 1] - P.sn_start[c];
                int32_t rc = P.sn_rowptr[c + 1] - P.sn_rowptr[c] - wc;
                for (int32_t a = 0; a < rc; ++a) {
                    int32_t src = P.sn_rowptr[c] + wc + a;
                    int32_t at = fill[P.sn_rowptr[p] + P.relmap[src]]++;
                    P.cb_src[at] = src;
                    P.cb_len[at] = rc - a;
                    P.cb_uoff[at] = P.u_off[c] + (int64_t)a * P.u_ld[c] + a;
                }
            }
    }

    // ---- levels (0 = leaves)
    std::vector<int32_t> lev(ns, 0);
    int32_t nlev = ns ? 1 : 0;
    for (int32_t s = 0; s < ns; ++s) {
        if (P.sn_parent[s] >= 0) lev[P.sn_parent[s]] = std::max(lev[P.sn_parent[s]], lev[s] + 1);
        nlev = std::max(nlev, lev[s] + 1);
    }
    P.nlev = nlev;
    P.sn_level = lev;
    auto group_by_level = [&](auto pred, std::vector<int32_t>& ptr, std::vector<int32_t>& list) {
        ptr.assign(nlev + 1, 0);
        for (int32_t s = 0; s < ns; ++s)
            if (pred(s)) ptr[lev[s] + 1]++;
        for (int32_t l = 0; l < nlev; ++l) ptr[l + 1] += ptr[l];
        list.resize(ptr[nlev]);
        std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
        for (int32_t s = 0; s < ns; ++s)
            if (pred(s)) list[fill[lev[s]]++] = s;
    };
    group_by_level([&](int32_t s) { return !P.big[s]; }, P.lvl_small_ptr, P.lvl_small);
    // small fronts of a level in increasing front order, so that one launch
    // per LDS size class covers a contiguous range
    for (int32_t l = 0; l < nlev; ++l)
        std::stable_sort(P.lvl_small.begin() + P.lvl_small_ptr[l], P.lvl_small.begin() + P.lvl_small_ptr[l + 1],
                         [&](int32_t x, int32_t y) {
                             return P.sn_rowptr[x + 1] - P.sn_rowptr[x] < P.sn_rowptr[y + 1] - P.sn_rowptr[y];
                         });
    group_by_level([&](int32_t s) { return P.big[s] != 0; }, P.lvl_big_ptr, P.lvl_big);
    group_by_level([&](int32_t) { return true; }, P.lvl_all_ptr, P.lvl_all);
    P.lvl_maxw_big.assign(nlev, 0);
    P.big_tiles_ptr.assign(nlev + 1, 0);
    P.big_tile_sn.clear();
    P.big_tile_col.clear();
    for (int32_t l = 0; l < nlev; ++l) {
        for (int32_t t = P.lvl_big_ptr[l]; t < P.lvl_big_ptr[l + 1]; ++t) {
            int32_t s = P.lvl_big[t];
            int32_t w = P.sn_start[s + 1] - P.sn_start[s];
            int32_t f = P.sn_rowptr[s + 1] - P.sn_rowptr[s];
            P.lvl_maxw_big[l] = std::max(P.lvl_maxw_big[l], w);
            for (int32_t c = 0; c < f; c += o.tile) {
                P.big_tile_sn.push_back(s);
                P.big_tile_col.push_back(c);
            }
        }
        P.big_tiles_ptr[l + 1] = (int32_t)P.big_tile_sn.size();
    }

    // ---- assembly recipe
    auto slot_of = [&](int32_t I, int32_t J) -> int32_t {  // I >= J, new numbering
        auto b = P.krow.begin() + P.kcolptr[J], e = P.krow.begin() + P.kcolptr[J + 1];
        auto it = std::lower_bound(b, e, I);
        if (it == e || *it != I) return -1;
        return (int32_t)(it - P.krow.begin());
    };
    P.k_wsrc.assign(nnzk, -1);
    P.k_diag.assign(nnzk, -1);
    for (int32_t j = 0; j < n; ++j) P.k_diag[P.kcolptr[j]] = P.perm[j];
    for (int32_t i = 0; i < n; ++i)
        for (int32_t k = p.w_ptr[i]; k < p.w_ptr[i + 1]; ++k) {
            int32_t I = P.iperm[i], J = P.iperm[p.w_idx[k]];
            int32_t sl = slot_of(std::max(I, J), std::min(I, J));
            if (sl < 0) return "internal: W entry missing from K";
            P.k_wsrc[sl] = k;
        }
    ts = std::chrono::steady_clock::now();
    err = o.device ? o.device->products(P, dense) : products_host(P, dense, o.threads);
    P.symbolic_seconds += since(ts);
    if (!err.empty()) return err;

    // ---- unassembled operators (original numbering)
    {
        P.wf_ptr.assign(n + 1, 0);
        for (int32_t i = 0; i < n; ++i)
            for (int32_t k = p.w_ptr[i]; k < p.w_ptr[i + 1]; ++k) {
                P.wf_ptr[i + 1]++;
                if (p.w_idx[k] != i) P.wf_ptr[p.w_idx[k] + 1]++;
            }
        for (int32_t i = 0; i < n; ++i) P.wf_ptr[i + 1] += P.wf_ptr[i];
        P.wf_col.resize(P.wf_ptr[n]);
        P.wf_vidx.resize(P.wf_ptr[n]);
        std::vector<int32_t> fill(P.wf_ptr.begin(), P.wf_ptr.end() - 1);
        // Row j of the full W: its own lower entries (columns <= j, strictly
        // increasing, as validate() checks) are written when row j is
        // visited, then the entries (i, j) of the rows i > j in increasing i:
        // every row comes out sorted without a sort.
        for (int32_t i = 0; i < n; ++i)
            for (int32_t k = p.w_ptr[i]; k < p.w_ptr[i + 1]; ++k) {
                int32_t j = p.w_idx[k];
                P.wf_col[fill[i]] = j; P.wf_vidx[fill[i]++] = k;
                if (j != i) { P.wf_col[fill[j]] = i; P.wf_vidx[fill[j]++] = k; }
            }
    }
    {
        P.jt_ptr.assign(n + 1, 0);
        for (int64_t a = 0; a < (int64_t)P.j_col.size(); ++a) P.jt_ptr[P.j_col[a] + 1]++;
        for (int32_t i = 0; i < n; ++i) P.jt_ptr[i + 1] += P.jt_ptr[i];
        P.jt_row.resize(P.j_col.size());
        P.jt_vidx.resize(P.j_col.size());
        std::vector<int32_t> fill(P.jt_ptr.begin(), P.jt_ptr.end() - 1);
        for (int32_t r = 0; r < m; ++r)  // rows increasing: G rows first in every column
            for (int32_t a = P.j_ptr[r]; a < P.j_ptr[r + 1]; ++a) {
                int32_t c = P.j_col[a];
                P.jt_row[fill[c]] = r;
                P.jt_vidx[fill[c]++] = a;
            }
        P.jt_gend.resize(n);
        for (int32_t i = 0; i < n; ++i) {
            int32_t t = P.jt_ptr[i];
            while (t < P.jt_ptr[i + 1] && P.jt_row[t] < P.m_eq) ++t;
            P.jt_gend[i] = t;
        }
    }
    if (P.inst_n.empty()) {
        P.ninst = 1;
        P.inst_n = {0, n};
        P.inst_meq = {0, P.m_eq};
        P.inst_of_var.assign(n, 0);
        P.inst_of_eqrow.assign(P.m_eq, 0);
    }
    P.analyze_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return "";
}

}  // namespace ckkt
