// Test-only cross-check: prints Philox4x32-10 blocks computed by the
// independent implementation in PyTorch's ATen/core/PhiloxRNGEngine.h.
// Reads lines "key_lo key_hi c0 c1 c2 c3" (decimal) from stdin and prints
// "o0 o1 o2 o3".  The engine keys by the 64-bit seed and counts by
// (offset_lo, offset_hi, subsequence_lo, subsequence_hi), so a counter
// (c0, c1, c2, c3) is offset = c0 | c1 << 32 and subsequence = c2 | c3 << 32.
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdint>
#include <cstdio>

int main() {
    unsigned long long klo, khi, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &klo, &khi, &c0, &c1, &c2, &c3) == 6) {
        uint64_t seed = (uint64_t)klo | ((uint64_t)khi << 32);
        uint64_t subseq = (uint64_t)c2 | ((uint64_t)c3 << 32);
        uint64_t offset = (uint64_t)c0 | ((uint64_t)c1 << 32);
        at::Philox4_32 eng(seed, subseq, offset);
        uint32_t o0 = eng(), o1 = eng(), o2 = eng(), o3 = eng();
        std::printf("%u %u %u %u\n", o0, o1, o2, o3);
    }
    return 0;
}
