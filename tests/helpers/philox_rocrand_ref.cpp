// Prints rocRAND's Philox4x32-10 output for (counter, key) lines read from
// stdin: "c0 c1 c2 c3 k0 k1" (hex).  Uses the library's header-only engine
// on the host; its seed(seed, subsequence, offset) places the counter at
// (offset/4 low/high words, subsequence low/high words).
#include <cstdio>
#include <cstdint>
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>

int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
        unsigned long long subseq = ((unsigned long long)c3 << 32) | c2;
        unsigned long long offset = (((unsigned long long)c1 << 32) | c0) * 4ull;
        rocrand_device::philox4x32_10_engine eng(seed, subseq, offset);
        unsigned a = eng.next(), b = eng.next(), c = eng.next(), d = eng.next();
        std::printf("%08x %08x %08x %08x\n", a, b, c, d);
    }
    return 0;
}
