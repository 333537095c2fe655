// Driver of the page-image store of streamed scenes for the CPU tests.
// Usage: page_store_harness <file|-> <n_pages> <page_bytes> <direct 0|1>
// Writes n_pages images (image k: byte i = (k * 131 + i * 7) mod 251), then
// reads the batches given on stdin ("get k0 k1 ...", ascending) and prints,
// per batch: ok tier reads_so_far | for each image whether it came back
// exactly and whether the slot padding after it is untouched (1 1 ...).
#include <cstdint>
#include <cstdlib>
#include <iostream>
#include <sstream>
#include <string>
#include <vector>

#include "page_store.h"

static uint8_t pattern(uint32_t k, uint64_t i) { return (uint8_t)((k * 131u + i * 7u) % 251u); }

int main(int argc, char **argv)
{
    if (argc != 5) return 2;
    const std::string path = argv[1];
    const uint32_t n = (uint32_t)std::atoi(argv[2]), pb = (uint32_t)std::atoi(argv[3]);
    const bool direct = std::atoi(argv[4]) != 0;
    v3dg::PageStore st;
    std::string err;
    if (path == "-") {
        st.init_memory(n, pb);
    } else if (!st.init_file(path.c_str(), n, pb, direct, false, &err)) {
        std::cout << "init failed " << err << "\n";
        return 1;
    }
    std::vector<uint8_t> img(pb);
    for (uint32_t k = 0; k < n; ++k) {
        for (uint32_t i = 0; i < pb; ++i) img[i] = pattern(k, i);
        if (!st.put(k, img.data(), &err)) {
            std::cout << "put failed " << err << "\n";
            return 1;
        }
    }
    if (!st.seal(&err)) {
        std::cout << "seal failed " << err << "\n";
        return 1;
    }
    std::cout << "ready " << st.tier() << ' ' << st.stride() << "\n" << std::flush;
    std::string line;
    while (std::getline(std::cin, line)) {
        std::istringstream is(line);
        std::string cmd;
        is >> cmd;
        std::vector<uint32_t> ks;
        uint32_t k;
        while (is >> k) ks.push_back(k);
        const uint64_t stride = st.stride();
        void *buf = nullptr;
        if (posix_memalign(&buf, 4096, (ks.size() + 1) * stride) != 0) return 1;
        uint8_t *dst = static_cast<uint8_t *>(buf);
        for (uint64_t i = 0; i < (ks.size() + 1) * stride; ++i) dst[i] = 0xAB;
        const bool ok = st.get(ks.data(), (uint32_t)ks.size(), dst, &err);
        std::cout << (ok ? 1 : 0) << ' ' << st.tier() << ' ' << st.reads() << " |";
        for (size_t j = 0; j < ks.size(); ++j) {
            bool same = true;
            for (uint32_t i = 0; i < pb; ++i) same = same && dst[j * stride + i] == pattern(ks[j], i);
            std::cout << ' ' << (same ? 1 : 0);
        }
        std::cout << " | " << (dst[ks.size() * stride] == 0xAB ? 1 : 0) << "\n" << std::flush;
        free(buf);
    }
    return 0;
}
