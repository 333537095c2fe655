// Line-driven driver of the page-replacement policy of streamed scenes, for
// the CPU tests: "init n_clusters n_pages", "plan k ...", "release k".
// plan prints: ok touched frame max_evicted_stamp evictions | misses | page of
// each miss | cluster of every page (-1: free).
#include <cstdint>
#include <iostream>
#include <sstream>
#include <string>
#include <vector>

#include "page_lru.h"

int main()
{
    v3dg::PageLRU lru;
    std::string line;
    while (std::getline(std::cin, line)) {
        std::istringstream is(line);
        std::string cmd;
        is >> cmd;
        if (cmd == "init") {
            uint32_t nc = 0, np = 0;
            is >> nc >> np;
            lru.init(nc, np);
            std::cout << "init\n";
        } else if (cmd == "plan") {
            std::vector<uint32_t> ks, miss;
            uint32_t k = 0, touched = 0;
            while (is >> k) ks.push_back(k);
            const bool ok = lru.plan(ks.data(), ks.size(), miss, touched);
            std::cout << (ok ? 1 : 0) << ' ' << touched << ' ' << lru.frame << ' ' << lru.max_evicted_stamp << ' '
                      << lru.evictions << " |";
            for (uint32_t m : miss) std::cout << ' ' << m;
            std::cout << " |";
            for (uint32_t m : miss) std::cout << ' ' << lru.page_of(m);
            std::cout << " |";
            for (uint32_t p = 0; p < lru.n_pages(); ++p)
                std::cout << ' ' << (lru.cluster_of(p) == v3dg::PageLRU::kNone ? -1 : (int64_t)lru.cluster_of(p));
            std::cout << '\n';
        } else if (cmd == "release") {
            uint32_t k = 0;
            is >> k;
            lru.release(k);
            std::cout << "release\n";
        }
        std::cout.flush();
    }
    return 0;
}
