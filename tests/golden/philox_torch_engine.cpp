// Prints the first four 32-bit outputs of PyTorch's open-source Philox4x32-10
// engine (ATen/core/PhiloxRNGEngine.h) for a given (seed, subsequence, offset).
// That engine sets key = (seed lo, seed hi) and
// counter = (offset lo, offset hi, subsequence lo, subsequence hi), so the
// four words are Philox4x32-10(counter, key): an implementation independent
// of the oracle's, used only by the CPU tests to pin the oracle's stream.
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cstdlib>

int main(int argc, char** argv) {
  for (int a = 1; a + 2 < argc; a += 3) {
    unsigned long long seed = strtoull(argv[a], 0, 0);
    unsigned long long sub = strtoull(argv[a + 1], 0, 0);
    unsigned long long off = strtoull(argv[a + 2], 0, 0);
    at::Philox4_32 e(seed, sub, off);
    for (int i = 0; i < 4; ++i) printf("%u ", (unsigned)e());
    printf("\n");
  }
  return 0;
}
