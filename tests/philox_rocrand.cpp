// Test helper: prints rocRAND's Philox4x32-10 output block for each
// "c0 c1 c2 c3 k0 k1" line on stdin.  rocRAND is an independent
// implementation of the same generator; its engine places the 64-bit seed in
// the key and (offset / 4, subsequence) in the counter words, so the block of
// counter (c0, c1, c2, c3) is reached with offset = 4 (c0 | c1 << 32) and
// subsequence = c2 | c3 << 32.  Host code only.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    unsigned long long seed = k0 | (static_cast<unsigned long long>(k1) << 32);
    unsigned long long subseq = c2 | (static_cast<unsigned long long>(c3) << 32);
    unsigned long long offset = 4ULL * (c0 | (static_cast<unsigned long long>(c1) << 32));
    rocrand_device::philox4x32_10_engine e(seed, subseq, offset);
    unsigned w0 = e.next(), w1 = e.next(), w2 = e.next(), w3 = e.next();
    std::printf("%u %u %u %u\n", w0, w1, w2, w3);
  }
  return 0;
}
