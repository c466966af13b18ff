// Known-answer generator for the Philox4x32-10 pin: runs PyTorch's own
// open-source Philox engine (ATen/core/PhiloxRNGEngine.h), an implementation
// independent of both the oracle and the HIP path.  Reads lines
// "c0 c1 c2 c3 seed" and prints the block "w0 w1 w2 w3".  PyTorch's engine
// keeps (offset_lo, offset_hi, subsequence_lo, subsequence_hi) as the
// counter and the seed as the key, so one block is four calls.
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdint>
#include <cstdio>

int main() {
  unsigned long long c0, c1, c2, c3, seed;
  while (std::scanf("%llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &seed) == 5) {
    at::philox_engine e(seed, (uint64_t)c2 | ((uint64_t)c3 << 32),
                        (uint64_t)c0 | ((uint64_t)c1 << 32));
    unsigned w0 = e(), w1 = e(), w2 = e(), w3 = e();
    std::printf("%u %u %u %u\n", w0, w1, w2, w3);
  }
  return 0;
}
