// Stress driver for the served form's host copy pool: several threads call
// run() at once with random copy lists (sizes 0 to a few MB, so long copies
// are cut and shared out), and every destination is checked byte for byte.
// Built with ThreadSanitizer or AddressSanitizer by the CPU tests.
#include <cstdint>
#include <cstdio>
#include <random>
#include <thread>
#include <vector>

#include "copy_pool.h"

int main(int argc, char** argv) {
  const int pool_threads = argc > 1 ? std::atoi(argv[1]) : 4;
  const int callers = argc > 2 ? std::atoi(argv[2]) : 3;
  const int rounds = argc > 3 ? std::atoi(argv[3]) : 40;
  bm::CopyPool pool(pool_threads);
  std::vector<int> bad(callers, 0);
  std::vector<std::thread> th;
  for (int c = 0; c < callers; ++c)
    th.emplace_back([&, c] {
      std::mt19937_64 rng(1234 + c);
      for (int r = 0; r < rounds; ++r) {
        const int k = (int)(rng() % 12);
        std::vector<std::vector<uint8_t>> src(k), dst(k);
        std::vector<bm::CopyPool::Copy> copies;
        for (int i = 0; i < k; ++i) {
          const size_t n = (rng() % 4 == 0) ? (size_t)(rng() % (3u << 20)) : (size_t)(rng() % 5000);
          src[i].resize(n);
          for (size_t b = 0; b < n; ++b) src[i][b] = (uint8_t)(b * 131 + i * 7 + r + c);
          dst[i].assign(n, 0xEE);
          copies.push_back(bm::CopyPool::Copy{src[i].data(), dst[i].data(), n});
        }
        pool.run(copies);
        for (int i = 0; i < k; ++i)
          if (src[i] != dst[i]) ++bad[c];
      }
    });
  for (auto& t : th) t.join();
  int total = 0;
  for (int b : bad) total += b;
  std::printf("copy pool: %d threads, %d callers x %d rounds, %d wrong copies\n", pool_threads, callers, rounds, total);
  return total == 0 ? 0 : 1;
}
