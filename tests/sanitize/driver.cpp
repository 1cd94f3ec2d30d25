// Host-side driver for the sanitizer builds of the analysis and of the
// sequential host factor-solve: reads patterns and values written by the
// test, analyses each (with several threads for the assembly recipe), runs
// the host factor-solve and prints one line per case.  Built with g++ only.
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "analysis.hpp"

namespace ckkt {
int host_factor_solve(const Plan& P, int hy, const double* w_val, const double* g_val, const double* h_val,
                      const double* sigma_x, const double* sigma_s, double gamma, const double* b, double* x);
}

using namespace ckkt;

template <typename T>
static bool rd(FILE* f, std::vector<T>& v) {
    long long n = 0;
    if (std::fread(&n, sizeof n, 1, f) != 1 || n < 0) return false;
    v.resize((size_t)n);
    return n == 0 || std::fread(v.data(), sizeof(T), (size_t)n, f) == (size_t)n;
}

int main(int argc, char** argv) {
    if (argc < 2) return 2;
    FILE* f = std::fopen(argv[1], "rb");
    if (!f) return 2;
    int cases = 0;
    for (;;) {
        std::vector<int32_t> head;
        if (!rd(f, head)) break;
        if (head.size() != 5) return 3;
        PatternIn p;
        std::vector<double> w, g, h, sx, ss, b;
        bool ok = rd(f, p.w_ptr) && rd(f, p.w_idx) && rd(f, p.g_ptr) && rd(f, p.g_idx) && rd(f, p.h_ptr) &&
                  rd(f, p.h_idx) && rd(f, w) && rd(f, g) && rd(f, h) && rd(f, sx) && rd(f, ss) && rd(f, b);
        if (!ok) return 3;
        p.n = head[0];
        p.m_eq = head[1];
        p.m_ineq = head[2];
        const int hy = head[3];
        AnalyzeOptions o;
        o.dense_row_min = head[4];
        o.threads = 4;
        Plan P;
        std::string err = analyze(p, o, P);
        if (!err.empty()) {
            std::printf("case %d analyze error %s\n", cases, err.c_str());
            return 4;
        }
        std::vector<double> x(b.size());
        const int fc = host_factor_solve(P, hy, w.data(), g.data(), h.data(), sx.data(), ss.data(), 1e7, b.data(),
                                         x.data());
        double sum = 0.0;
        for (double v : x) sum += v;
        std::printf("case %d n %lld nnz_l %lld dense %zu failed %d sum %.6e\n", cases, (long long)p.n,
                    (long long)P.nnz_l, P.dense_rows.size(), fc, sum);
        ++cases;
    }
    std::fclose(f);
    return cases > 0 ? 0 : 5;
}
