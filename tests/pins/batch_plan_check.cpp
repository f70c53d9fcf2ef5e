// Driver for the CPU checks of the batch engine's host planning
// (paper_2202_01753_amd/csrc/batch_plan.hpp).  Reads one command block from
// standard input and prints the result:
//   split <n> <parts>  then n lines "<m> <cost>"  ->  "piece <item> <t0> <t1>" lines,
//                                                     then "first <i> <index>" lines
//   order <n>          then n lines "<item> <t0> <t1> <cost>" -> one line of indices
//   arena <cap> <k>    then k lines "a <bytes>" or "r <off> <bytes>" -> one line per op
//                      ("ok <off>", "fail", "released"), then "free <bytes> <ranges>"
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
    } else {
        return 2;
    }
    return 0;
}
