// Independent Philox4x32-10 reference for the tests: PyTorch's header-only
// philox_engine (key = seed, counter words 0-1 = offset, 2-3 = subsequence).
// Reads "seed subsequence offset" triples from stdin and prints the 4 words.
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>

int main() {
    unsigned long long seed, sub, off;
    while (std::scanf("%llu %llu %llu", &seed, &sub, &off) == 3) {
        at::philox_engine e(seed, sub, off);
        unsigned w0 = e(), w1 = e(), w2 = e(), w3 = e();
        std::printf("%u %u %u %u\n", w0, w1, w2, w3);
    }
    return 0;
}
