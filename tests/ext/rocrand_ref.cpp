// Independent reference outputs for the two PRNG definitions, taken from the
// rocRAND device/host headers (an external library, not part of this
// project).  Used only by the CPU tests that pin the oracle's generators.
//
//   rocrand_ref philox c0 c1 c2 c3 k0 k1   -> four output words
//   rocrand_ref mrg seed site n             -> n outputs of MRG32k3a started
//                                              from (seed x 6) and advanced by
//                                              site * 2^127 steps
#include <rocrand/rocrand_kernel.h>
#include <cstdio>
#include <cstdlib>
#include <cstring>

struct mrg_access : rocrand_device::mrg32k3a_engine {
    void set_all(unsigned int s) {
        for (int k = 0; k < 3; ++k) { m_state.g1[k] = s; m_state.g2[k] = s; }
    }
    void jump_sequences(unsigned long long n) { discard_sequence(n); }
};

int main(int argc, char** argv) {
    if (argc >= 8 && !std::strcmp(argv[1], "philox")) {
        unsigned long long c[4], k[2];
        for (int i = 0; i < 4; ++i) c[i] = std::strtoull(argv[2 + i], nullptr, 0);
        for (int i = 0; i < 2; ++i) k[i] = std::strtoull(argv[6 + i], nullptr, 0);
        rocrand_state_philox4x32_10 st;
        unsigned long long seed = k[0] | (k[1] << 32);
        unsigned long long subseq = c[2] | (c[3] << 32);
        rocrand_init(seed, subseq, 0, &st);
        // advance the low 64 counter bits: discard(4 * 2^b) moves the counter by 2^b
        unsigned long long lo = c[0] | (c[1] << 32);
        if (lo >> 62) { std::fprintf(stderr, "low counter too large\n"); return 2; }
        for (int b = 0; b < 62; ++b)
            if ((lo >> b) & 1ull) st.discard(4ull << b);
        uint4 o = rocrand4(&st);
        std::printf("%u %u %u %u\n", o.x, o.y, o.z, o.w);
        return 0;
    }
    if (argc >= 5 && !std::strcmp(argv[1], "mrg")) {
        unsigned int s = (unsigned int)std::strtoull(argv[2], nullptr, 0);
        unsigned long long site = std::strtoull(argv[3], nullptr, 0);
        int n = std::atoi(argv[4]);
        mrg_access e;
        e.set_all(s);
        e.jump_sequences(site);
        for (int i = 0; i < n; ++i) std::printf("%u%c", e.next(), i + 1 < n ? ' ' : '\n');
        return 0;
    }
    std::fprintf(stderr, "usage\n");
    return 2;
}
