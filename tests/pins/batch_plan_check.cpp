// Driver for the CPU checks of the batch engine's host planning
// (paper_2202_01753_amd/csrc/batch_plan.hpp).  Reads one command block from
// standard input and prints the result:
//   split <n> <parts>  then n lines "<m> <cost>"  ->  "piece <item> <t0> <t1>" lines,
//                                                     then "first <i> <index>" lines
//   order <n>          then n lines "<item> <t0> <t1> <cost>" -> one line of indices
//   arena <cap> <k>    then k lines "a <bytes>" or "r <off> <bytes>" -> one line per op
//                      ("ok <off>", "fail", "released"), then "free <bytes> <ranges>"
//   select <n> <budget> <max_skip>  then n lines "<work> <samples> <skipped> <id>"
//                                   -> one line of 0/1 per candidate
//   iters <k>          then k lines "<it> <itmax> <tau> <estimate> <error>" -> one value per line
#include <cstdio>
#include <iostream>
#include <string>
#include <vector>

#include "batch_plan.hpp"

using namespace mcubes::plan;

int main() {
    std::string cmd;
    std::cin >> cmd;
    if (cmd == "split") {
        int n;
        long long parts;
        std::cin >> n >> parts;
        std::vector<int64_t> m(n);
        std::vector<double> cost(n);
        for (int i = 0; i < n; ++i) std::cin >> m[i] >> cost[i];
        std::vector<Piece> out;
        std::vector<int32_t> first(n, -1);
        split_work(m.data(), cost.data(), 0, n, parts, out, first.data());
        for (const Piece &p : out) std::printf("piece %d %lld %lld\n", p.item, (long long)p.t0, (long long)p.t1);
        for (int i = 0; i < n; ++i) std::printf("first %d %d\n", i, first[i]);
    } else if (cmd == "order") {
        int n;
        std::cin >> n;
        std::vector<Piece> pieces(n);
        std::vector<double> cost(n);
        for (int k = 0; k < n; ++k) {
            long long t0, t1;
            std::cin >> pieces[k].item >> t0 >> t1 >> cost[k];
            pieces[k].t0 = t0;
            pieces[k].t1 = t1;
        }
        // costs are indexed by item: here item k has the cost read on line k
        std::vector<int32_t> order;
        largest_first(pieces, cost.data(), 0, n, order);
        for (int32_t o : order) std::printf("%d ", o);
        std::printf("\n");
    } else if (cmd == "arena") {
        size_t cap;
        int k;
        std::cin >> cap >> k;
        Arena a(cap);
        for (int i = 0; i < k; ++i) {
            std::string op;
            std::cin >> op;
            if (op == "a") {
                size_t bytes, off = 0;
                std::cin >> bytes;
                if (a.alloc(bytes, &off)) std::printf("ok %zu\n", off);
                else std::printf("fail\n");
            } else {
                size_t off, bytes;
                std::cin >> off >> bytes;
                a.release(off, bytes);
                std::printf("released\n");
            }
        }
        std::printf("free %zu %zu\n", a.free_bytes(), a.free_ranges());
    } else if (cmd == "select") {
        int n, max_skip;
        long long budget;
        std::cin >> n >> budget >> max_skip;
        std::vector<Candidate> c(n);
        for (int i = 0; i < n; ++i) {
            long long samples, id;
            std::cin >> c[i].work >> samples >> c[i].skipped >> id;
            c[i].samples = samples;
            c[i].id = id;
        }
        const std::vector<char> run = select_for_step(c, budget, max_skip);
        for (int i = 0; i < n; ++i) std::printf("%d%s", (int)run[i], i + 1 < n ? " " : "\n");
    } else if (cmd == "iters") {
        int k;
        std::cin >> k;
        for (int i = 0; i < k; ++i) {
            int it, itmax;
            double tau, est, err;
            std::cin >> it >> itmax >> tau >> est >> err;
            std::printf("%.17g\n", expected_iterations(it, itmax, tau, est, err));
        }
    } else {
        return 2;
    }
    return 0;
}
