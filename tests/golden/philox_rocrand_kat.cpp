// Independent Philox4x32-10 reference for the oracle's known-answer test:
// rocRAND's open-source engine (header only, compiled for the host).
// Input lines on stdin: c0 c1 c2 c3 k0 k1 (decimal); output: w0 w1 w2 w3.
// The counter is reached through the public engine API: the 64-bit key is the
// seed, the upper counter half is the subsequence and the lower half times 4 the
// offset (each counter value yields four 32-bit outputs).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdint>

int main() {
    unsigned long long c0, c1, c2, c3, k0, k1;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = k0 | (k1 << 32);
        unsigned long long subseq = c2 | (c3 << 32);
        unsigned long long offset = 4ull * (c0 | (c1 << 32));
        rocrand_device::philox4x32_10_engine eng(seed, subseq, offset);
        unsigned int w0 = eng(), w1 = eng(), w2 = eng(), w3 = eng();
        std::printf("%u %u %u %u\n", w0, w1, w2, w3);
    }
    return 0;
}
