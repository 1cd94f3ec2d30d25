// Approximate minimum degree ordering on the quotient graph.
//
// Written from the published description of the method (Amestoy, Davis,
// Duff, SIAM J. Matrix Anal. Appl. 17(4), 1996): eliminated pivots become
// elements, each remaining variable keeps a variable list A_i and an
// element list E_i, the external degree is bounded from above by
//   min(n - k, d_i + |L_p \ i|, |A_i| + |L_p \ i| + sum_{e in E_i, e != p} |L_e \ L_p|)
// with |L_e \ L_p| obtained by one sweep over the new element, elements
// whose variables all lie in the new element are absorbed (aggressive
// absorption), and variables with identical adjacency are merged into
// supervariables (hash, then exact comparison).  The paper's CPU solver
// orders the condensed matrix with AMD (Sec. 5, CHOLMOD) -- this is our own
// implementation of that algorithm, used by the host analysis.
#include <algorithm>
#include <cstdint>
#include <numeric>
#include <vector>

#include "analysis.hpp"

namespace ckkt {

namespace {
enum : uint8_t { VAR = 0, ELEM = 1, DEAD = 2 };
}

std::vector<int32_t> amd_order(const Graph& g) {
    const int32_t n = g.n;
    std::vector<std::vector<int32_t>> A(n), E(n), Le(n);
    for (int32_t i = 0; i < n; ++i) A[i].assign(g.adj.begin() + g.ptr[i], g.adj.begin() + g.ptr[i + 1]);

    std::vector<int32_t> nv(n, 1), superp(n, -1), mark(n, -1), wst(n, -1);
    std::vector<int64_t> deg(n), degE(n, 0), w(n, 0), ext(n, 0);
    std::vector<uint64_t> hsh(n, 0);
    std::vector<uint8_t> st(n, VAR);

    // degree buckets: doubly linked lists
    std::vector<int32_t> head(n + 1, -1), nxt(n, -1), prv(n, -1);
    int64_t mindeg = n;
    auto insert = [&](int32_t i) {
        int64_t d = deg[i];
        nxt[i] = head[d];
        prv[i] = -1;
        if (head[d] >= 0) prv[head[d]] = i;
        head[d] = i;
        if (d < mindeg) mindeg = d;
    };
    auto remove = [&](int32_t i) {
        if (prv[i] >= 0) nxt[prv[i]] = nxt[i];
        else head[deg[i]] = nxt[i];
        if (nxt[i] >= 0) prv[nxt[i]] = prv[i];
        nxt[i] = prv[i] = -1;
    };
    for (int32_t i = 0; i < n; ++i) {
        deg[i] = (int64_t)A[i].size();
        insert(i);
    }

    std::vector<int32_t> order;
    order.reserve(n);
    std::vector<int32_t> Lp;
    int64_t nel = 0;
    while (nel < n) {
        while (mindeg <= n && head[mindeg] < 0) ++mindeg;
        const int32_t p = head[mindeg];
        remove(p);
        order.push_back(p);
        nel += nv[p];

        // ---- form the new element L_p = (A_p U union of L_e, e in E_p) \ {p}
        Lp.clear();
        mark[p] = p;
        for (int32_t e : E[p]) {
            if (st[e] != ELEM) continue;
            for (int32_t i : Le[e])
                if (st[i] == VAR && nv[i] > 0 && mark[i] != p) { mark[i] = p; Lp.push_back(i); }
            st[e] = DEAD;  // absorbed into p
            std::vector<int32_t>().swap(Le[e]);
        }
        for (int32_t i : A[p])
            if (st[i] == VAR && nv[i] > 0 && mark[i] != p) { mark[i] = p; Lp.push_back(i); }
        std::vector<int32_t>().swap(A[p]);
        std::vector<int32_t>().swap(E[p]);
        st[p] = ELEM;
        int64_t degLp = 0;
        for (int32_t i : Lp) { degLp += nv[i]; remove(i); }

        // ---- |L_e \ L_p| for every element touching L_p
        for (int32_t i : Lp)
            for (int32_t e : E[i]) {
                if (st[e] != ELEM || e == p) continue;
                if (wst[e] != p) { wst[e] = p; w[e] = degE[e]; }
                w[e] -= nv[i];
            }

        // ---- prune lists, external degree bound, hash
        for (int32_t i : Lp) {
            int64_t dext = 0;
            uint64_t h = 0;
            auto& Ei = E[i];
            size_t ke = 0;
            for (size_t t = 0; t < Ei.size(); ++t) {
                int32_t e = Ei[t];
                if (st[e] != ELEM || e == p) continue;
                int64_t we = w[e];
                if (we > 0) { dext += we; Ei[ke++] = e; h += (uint64_t)e * 0x9E3779B97F4A7C15ull; }
                else { st[e] = DEAD; std::vector<int32_t>().swap(Le[e]); }  // aggressive absorption
            }
            Ei.resize(ke);
            Ei.push_back(p);
            h += (uint64_t)p * 0x9E3779B97F4A7C15ull;
            auto& Ai = A[i];
            size_t ka = 0;
            for (size_t t = 0; t < Ai.size(); ++t) {
                int32_t j = Ai[t];
                if (st[j] != VAR || nv[j] == 0 || mark[j] == p || j == p) continue;
                Ai[ka++] = j;
                dext += nv[j];
                h += (uint64_t)j * 0xC2B2AE3D27D4EB4Full + 1;
            }
            Ai.resize(ka);
            ext[i] = dext;
            hsh[i] = h;
        }

        // ---- supervariable detection inside L_p
        if (Lp.size() > 1) {
            std::vector<int32_t> cand(Lp);
            std::sort(cand.begin(), cand.end(), [&](int32_t a, int32_t b) {
                if (hsh[a] != hsh[b]) return hsh[a] < hsh[b];
                return a < b;
            });
            size_t s0 = 0;
            while (s0 < cand.size()) {
                size_t s1 = s0 + 1;
                while (s1 < cand.size() && hsh[cand[s1]] == hsh[cand[s0]]) ++s1;
                if (s1 - s0 > 1) {
                    for (size_t a = s0; a < s1; ++a) {
                        std::sort(A[cand[a]].begin(), A[cand[a]].end());
                        std::sort(E[cand[a]].begin(), E[cand[a]].end());
                    }
                    for (size_t a = s0; a < s1; ++a) {
                        int32_t i = cand[a];
                        if (nv[i] == 0) continue;
                        for (size_t b = a + 1; b < s1; ++b) {
                            int32_t j = cand[b];
                            if (nv[j] == 0) continue;
                            if (A[i] == A[j] && E[i] == E[j]) {
                                nv[i] += nv[j];
                                nv[j] = 0;
                                st[j] = DEAD;
                                superp[j] = i;
                                std::vector<int32_t>().swap(A[j]);
                                std::vector<int32_t>().swap(E[j]);
                            }
                        }
                    }
                }
                s0 = s1;
            }
        }

        // ---- degree update and the new element's list
        std::vector<int32_t> keep;
        keep.reserve(Lp.size());
        const int64_t rem = (int64_t)n - nel;
        for (int32_t i : Lp) {
            if (nv[i] == 0) continue;
            keep.push_back(i);
            int64_t other = degLp - nv[i];
            int64_t d = std::min({rem - nv[i], deg[i] + other, ext[i] + other});
            if (d < 0) d = 0;
            if (d > n) d = n;
            deg[i] = d;
            insert(i);
        }
        degE[p] = degLp;
        Le[p].swap(keep);
    }

    // ---- expand supervariables: members follow their principal pivot
    std::vector<std::vector<int32_t>> members(n);
    for (int32_t j = 0; j < n; ++j) {
        if (superp[j] < 0) continue;
        int32_t r = j;
        while (superp[r] >= 0) r = superp[r];
        members[r].push_back(j);
    }
    std::vector<int32_t> perm;
    perm.reserve(n);
    for (int32_t p : order) {
        perm.push_back(p);
        for (int32_t j : members[p]) perm.push_back(j);
    }
    return perm;
}

}  // namespace ckkt
