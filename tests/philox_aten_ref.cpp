// Reads lines "c0 c1 c2 c3 k0 k1" and prints the four Philox4x32-10 words
// produced by PyTorch's independent header-only engine (ATen).  Used only to
// pin the oracle's Philox; it is compiled by the test, never linked anywhere.
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>

int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        const uint64_t seed = (uint64_t)k0 | ((uint64_t)k1 << 32);
        const uint64_t sub = (uint64_t)c2 | ((uint64_t)c3 << 32);
        const uint64_t off = (uint64_t)c0 | ((uint64_t)c1 << 32);
        at::Philox4_32 e(seed, sub, off);
        const unsigned a = e(), b = e(), c = e(), d = e();
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
