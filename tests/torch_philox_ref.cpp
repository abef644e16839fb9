// Prints Philox4x32-10 output words from PyTorch's header-only engine (an independent implementation)
// for (seed, subsequence, offset) triples read from stdin, four words per triple.
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdint>
#include <cstdio>

int main() {
  unsigned long long seed, subseq, offset;
  while (std::scanf("%llu %llu %llu", &seed, &subseq, &offset) == 3) {
    at::philox_engine eng(seed, subseq, offset);
    for (int k = 0; k < 4; ++k) std::printf("%u ", (unsigned)eng());
    std::printf("\n");
  }
  return 0;
}
