// Raw Philox4x32-10 blocks from rocRAND's host/device engine, for pinning the oracle's generator against an
// independent implementation.  Reads lines "c0 c1 c2 c3 k0 k1" (hexadecimal) and prints the four output words.
// rocRAND's engine keeps the counter as (low 64 bits: position, high 64 bits: subsequence) and the key as the
// seed's two 32-bit halves, so a given counter is reached by seeding the subsequence and discarding the position.
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    while (scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        const unsigned long long key = (unsigned long long)k1 << 32 | k0;
        const unsigned long long lo = (unsigned long long)c1 << 32 | c0, hi = (unsigned long long)c3 << 32 | c2;
        rocrand_device::philox4x32_10_engine e(key, hi, 0);
        for (int i = 0; i < 4; ++i) e.discard(lo);   // four quarter steps add lo to the counter, substate back to 0
        const unsigned w0 = e(), w1 = e(), w2 = e(), w3 = e();
        printf("%08x %08x %08x %08x\n", w0, w1, w2, w3);
    }
    return 0;
}
