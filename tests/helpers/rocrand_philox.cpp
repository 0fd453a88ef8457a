// Test helper: prints rocRAND's Philox4x32-10 block for each (seed, s, d, tag)
// line on stdin, using the library's host-callable engine.  The engine's
// counter is (offset/4 low, high, subsequence low, high), so counter
// (s lo, s hi, d, tag) is subsequence d | tag<<32 at offset 4*s.
#include <rocrand/rocrand_kernel.h>
#include <cstdio>
int main() {
    unsigned long long seed, s;
    unsigned d, tag;
    while (scanf("%llu %llu %u %u", &seed, &s, &d, &tag) == 4) {
        rocrand_device::philox4x32_10_engine e(seed, (unsigned long long)d | ((unsigned long long)tag << 32),
                                               s * 4ULL);
        unsigned a = e.next(), b = e.next(), c = e.next(), w = e.next();
        printf("%u %u %u %u\n", a, b, c, w);
    }
    return 0;
}
