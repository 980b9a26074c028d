// Host-side cross-check of Philox4x32-10 against rocRAND's independent implementation.
// Reads lines "c0 c1 c2 c3 k0 k1" (decimal) from stdin, prints the four output words.
// Used only by the oracle's tests.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

// ten_rounds is a protected member: a derived class makes it callable.
struct philox_rounds : rocrand_device::philox4x32_10_engine {
    using rocrand_device::philox4x32_10_engine::ten_rounds;
};

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    philox_rounds eng;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 ctr = {c0, c1, c2, c3};
        uint2 key = {k0, k1};
        uint4 out = eng.ten_rounds(ctr, key);
        std::printf("%u %u %u %u\n", out.x, out.y, out.z, out.w);
    }
    return 0;
}
