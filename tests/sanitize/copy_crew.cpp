// The host copy crew (csrc/ss_copy.h) under ThreadSanitizer: six threads copy buffers of random
// sizes (below and above the size where the crew takes part, ragged last pieces) through one
// crew of three helpers at once, and every destination is compared byte for byte with its source.
// A second crew is destroyed while idle, and a crew without helpers copies alone.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <thread>
#include <vector>

#include "ss_copy.h"

int main()
{
    int bad = 0;
    {
        ss::CopyCrew crew(3);
        if (crew.helpers() != 3) {
            std::printf("helpers: %d\n", crew.helpers());
            return 1;
        }
        std::vector<std::thread> th;
        std::vector<int> errs(6, 0);
        for (int t = 0; t < 6; t++) {
            th.emplace_back([&, t] {
                std::mt19937_64 rng(1910090200 + t);
                for (int it = 0; it < 12; it++) {
                    const size_t sizes[] = {0, 1, 4095, ss::CopyCrew::kMin - 1, ss::CopyCrew::kMin,
                                            ss::CopyCrew::kMin + 12345, 5 * ss::CopyCrew::kPiece + 7};
                    const size_t n = sizes[rng() % (sizeof(sizes) / sizeof(sizes[0]))];
                    std::vector<uint8_t> src(n + 1), dst(n + 1, 0xEE);
                    for (size_t i = 0; i < n; i++) src[i] = (uint8_t)(rng() >> 7);
                    crew.copy(dst.data(), src.data(), n);
                    if (std::memcmp(dst.data(), src.data(), n) != 0 || dst[n] != 0xEE) errs[t]++;
                }
            });
        }
        for (auto& x : th) x.join();
        for (int e : errs) bad += e;
        ss::CopyCrew idle(2);                    // destroyed without work
        ss::CopyCrew alone(0);
        std::vector<uint8_t> a(3 << 20, 7), b(3 << 20, 0);
        alone.copy(b.data(), a.data(), a.size());
        bad += b != a;
    }
    if (bad) {
        std::printf("copy crew: %d wrong copies\n", bad);
        return 1;
    }
    std::printf("copy crew: ok\n");
    return 0;
}
