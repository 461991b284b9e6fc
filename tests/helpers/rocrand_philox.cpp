// Independent Philox4x32-10 reference for the oracle's CPU pin: rocRAND's
// host-callable engine (a library routine), driven through its public
// seed / subsequence / offset interface.  Reads lines "k0 k1 c0 c1 c2 c3"
// (decimal) and prints the four output words of that counter and key.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
    unsigned long long k0, k1, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        rocrand_state_philox4x32_10 st;
        unsigned long long seed = (k1 << 32) | k0;
        unsigned long long subsequence = (c3 << 32) | c2;  // counter words z, w
        unsigned long long offset = ((c1 << 32) | c0) * 4ULL; // counter words x, y
        rocrand_init(seed, subsequence, offset, &st);
        uint4 r = rocrand4(&st);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
