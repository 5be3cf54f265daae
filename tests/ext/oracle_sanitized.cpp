// The FP64 oracle driven through its C interface under AddressSanitizer and
// UndefinedBehaviorSanitizer (see test_sanitizers.py): both groups, every
// generator, sweeps with accept logs, link and state I/O, measurement, the
// single-link primitives and the O(N) model, on small lattices with ragged
// and degenerate extents.
#include <cmath>
#include <cstdio>
#include <vector>

#include "oracle.h"

static int failures = 0;
#define CHECK(cond)                                                              \
    do {                                                                         \
        if (!(cond)) {                                                           \
            std::fprintf(stderr, "CHECK failed at line %d: %s\n", __LINE__, #cond); \
            ++failures;                                                          \
        }                                                                        \
    } while (0)

int main() {
    orc_set_threads(2);
    const int shapes[3][4] = {{4, 4, 4, 4}, {2, 2, 2, 2}, {6, 4, 2, 8}};
    for (int group = 2; group <= 3; ++group)
        for (int rng = 0; rng < 4; ++rng)
            for (const auto& d : shapes) {
                const int start = (group == 3 && rng == ORC_RNG_CONST) ? ORC_COLD : ORC_HOT;
                orc_lattice* L = orc_create(group, d[0], d[1], d[2], d[3], group == 3 ? 5.7 : 2.3, 1, rng, 0.5,
                                            rng == 0 ? 5 : 11, 10, 3, start, rng == 1 ? 1 : 0);
                CHECK(L != nullptr);
                if (!L) continue;
                const int V = d[0] * d[1] * d[2] * d[3];
                const int nc = group == 3 ? 18 : 4;
                orc_enable_accept_log(L, 1);
                orc_sweep(L, 2, 1);
                std::vector<int8_t> log((size_t)2 * 4 * V * 3);
                CHECK(orc_get_accept_log(L, log.data(), (int64_t)log.size()) == (int64_t)log.size());
                double plaq[3], poly[2];
                orc_measure(L, plaq, poly);
                // |P| <= 1 up to rounding (the constant generator makes every link equal: P = 1)
                if (!(std::isfinite(plaq[0]) && std::fabs(plaq[0]) <= 1.0 + 1e-12))
                    std::fprintf(stderr, "SU(%d) rng %d %dx%dx%dx%d: P = %.17g\n", group, rng, d[0], d[1], d[2], d[3],
                                 plaq[0]);
                CHECK(std::isfinite(plaq[0]) && std::fabs(plaq[0]) <= 1.0 + 1e-12);
                std::vector<double> links((size_t)V * 4 * nc);
                orc_get_links(L, links.data());
                orc_set_links(L, links.data());
                std::vector<uint32_t> st((size_t)V * 6);
                (void)orc_get_mrg_states(L, st.data());
                std::vector<double> A((size_t)2 * group * group);
                orc_staple(L, V - 1, 3, A.data());
                orc_destroy(L);
            }
    CHECK(orc_create(3, 3, 4, 4, 4, 5.7, 0, 1, 0.5, 1, 10, 0, 1, 0) == nullptr);  // odd extent refused
    CHECK(orc_create(3, 4, 4, 4, 4, 5.7, 0, ORC_RNG_CONST, 0.5, 1, 10, 0, ORC_HOT, 0) == nullptr);
    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
    orc_philox4x32_10(ctr, key, out);
    uint32_t st[6];
    CHECK(orc_mrg_site_state(12345, 77, st) == 0);
    (void)orc_mrg_next(st);
    orc_mrg_advance_pow2(st, 40);
    std::vector<uint32_t> rl(500);
    orc_ranlux_raw(7, 500, 1, rl.data());
    uint32_t sv[2];
    orc_ranlux_standard_values(sv);
    CHECK(sv[0] == 7937952u && sv[1] == 9901578u);
    std::vector<double> u(4 * 11 + 2, 0.5);
    double x[4];
    int used = 0;
    (void)orc_kp_sample(13.8, 10, u.data(), x, &used);
    CHECK(used > 0 && used <= (int)u.size());
    const double U[18] = {1, 0, 0, 0, 0, 0, 0, 0, 1, 0, 0, 0, 0, 0, 0, 0, 1, 0};
    double Ar[18] = {2, 0, 0.1, 0, 0, 0, 0, 0, 2, 0, 0, 0, 0, 0, 0, 0, 2, 0}, Uo[18];
    (void)orc_update_link(3, 5.7, 10, 0, 1, U, Ar, u.data(), Uo);
    (void)orc_update_link(3, 5.7, 10, 1, 1, U, Ar, u.data(), Uo);
    for (int n = 1; n <= 4; ++n)
        for (int rng = 0; rng < 4; ++rng) {
            orc_on* F = orc_on_create(n, 4, 2, 2, 4, 0.3, 1.0, 0.1, 0.55, rng, 0.5, rng == 0 ? 3 : 9, 20, 1, 1);
            CHECK(F != nullptr);
            if (!F) continue;
            orc_on_sweep(F, 2);
            double obs[7];
            orc_on_measure(F, obs);
            std::vector<double> f((size_t)64 * n);
            orc_on_get_field(F, f.data());
            orc_on_set_field(F, f.data());
            std::vector<uint32_t> ms((size_t)64 * 6);
            (void)orc_on_get_mrg_states(F, ms.data());
            CHECK(orc_on_acceptance(F) >= 0.0);
            orc_on_destroy(F);
        }
    if (failures) {
        std::fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    std::printf("oracle under sanitizers: ok\n");
    return 0;
}
