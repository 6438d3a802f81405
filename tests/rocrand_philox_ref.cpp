// Reads "seed c0 c1 c2 c3" lines on stdin and prints rocRAND's Philox4x32-10
// output for that key and counter.  rocRAND's engine maps (seed, subsequence,
// offset) to key = seed and counter = (offset / 4 as c0|c1, subsequence as
// c2|c3), so each query is one rocrand_init + rocrand4.  Host-only use of the
// library's header; an independent implementation to pin the oracle against.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
    unsigned long long seed;
    unsigned int c0, c1, c2, c3;
    while (std::scanf("%llu %u %u %u %u", &seed, &c0, &c1, &c2, &c3) == 5) {
        unsigned long long subsequence = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        unsigned long long offset = 4ull * ((unsigned long long)c0 | ((unsigned long long)c1 << 32));
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, subsequence, offset, &st);
        uint4 v = rocrand4(&st);
        std::printf("%u %u %u %u\n", v.x, v.y, v.z, v.w);
    }
    return 0;
}
