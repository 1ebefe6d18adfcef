// Third, independent Philox4x32-10: the one shipped with rocRAND, used only
// through its public device/host API (rocrand_init + rocrand4).  rocRAND keys
// the block function with the 64-bit seed (low word first) and sets counter
// words 2,3 from the subsequence and words 0,1 from offset/4.
// Reads lines "c0 c1 c2 c3 k0 k1" (decimal) from stdin, prints the 4 outputs.
#include <rocrand_kernel.h>
#include <cstdio>
int main() {
    unsigned int c[4], k[2];
    while (std::scanf("%u %u %u %u %u %u", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
        unsigned long long seed = (unsigned long long)k[0] | ((unsigned long long)k[1] << 32);
        unsigned long long sub = (unsigned long long)c[2] | ((unsigned long long)c[3] << 32);
        unsigned long long cnt = (unsigned long long)c[0] | ((unsigned long long)c[1] << 32);
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, sub, 0, &st);
        // advance the counter by cnt blocks (4 outputs each) without forming 4*cnt
        for (int q = 0; q < 4; ++q) skipahead(cnt, &st);
        uint4 r = rocrand4(&st);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
