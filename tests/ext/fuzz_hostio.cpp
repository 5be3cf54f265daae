// CPU fuzzing of the library's host-side file formats, built with
// AddressSanitizer and UndefinedBehaviorSanitizer (see test_sanitizers.py):
// the SU(N) and O(N) checkpoint readers and the tuning-cache parser get
// valid files, every truncation, seeded random corruptions and crafted
// headers (consistent checksums, extreme sizes); every call must return a
// status without a sanitizer report, and only intact files may be accepted.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "lat_hostio.hpp"

using namespace lathost;

static int failures = 0;
#define CHECK(cond)                                                              \
    do {                                                                         \
        if (!(cond)) {                                                           \
            std::fprintf(stderr, "CHECK failed at line %d: %s\n", __LINE__, #cond); \
            ++failures;                                                          \
        }                                                                        \
    } while (0)

static std::vector<unsigned char> slurp(const std::string& p) {
    std::vector<unsigned char> v;
    FILE* f = std::fopen(p.c_str(), "rb");
    if (!f) return v;
    int c;
    while ((c = std::fgetc(f)) != EOF) v.push_back((unsigned char)c);
    std::fclose(f);
    return v;
}

static void spit(const std::string& p, const std::vector<unsigned char>& v) {
    FILE* f = std::fopen(p.c_str(), "wb");
    if (!f) std::abort();
    if (!v.empty()) std::fwrite(v.data(), 1, v.size(), f);
    std::fclose(f);
}

template <class H>
static ckpt_status read_any(const std::string& p, H& h, std::vector<double>& d, std::vector<uint32_t>& w);
template <>
ckpt_status read_any<su_header>(const std::string& p, su_header& h, std::vector<double>& d, std::vector<uint32_t>& w) {
    return read_su_checkpoint(p.c_str(), h, d, w);
}
template <>
ckpt_status read_any<on_header>(const std::string& p, on_header& h, std::vector<double>& d, std::vector<uint32_t>& w) {
    return read_on_checkpoint(p.c_str(), h, d, w);
}

// Writes a file whose checksum is correct for the given (possibly invalid)
// header, so that only the header checks stand between it and the reader.
template <class H>
static void write_with_checksum(const std::string& p, const H& h, size_t nd, size_t nw) {
    std::vector<double> d(nd, 0.25);
    std::vector<uint32_t> w(nw, 7u);
    CHECK(write_checkpoint(p.c_str(), &h, sizeof h, d.data(), nd, w.data(), nw));
}

template <class H>
static void fuzz_file(const std::string& p, const H& good, size_t nd, size_t nw, std::mt19937_64& rng) {
    std::vector<double> d0(nd);
    std::vector<uint32_t> w0(nw);
    for (size_t i = 0; i < nd; ++i) d0[i] = std::ldexp((double)(rng() >> 11), -53);
    for (size_t i = 0; i < nw; ++i) w0[i] = (uint32_t)rng();
    CHECK(write_checkpoint(p.c_str(), &good, sizeof good, d0.data(), nd, w0.data(), nw));
    H h;
    std::vector<double> d;
    std::vector<uint32_t> w;
    CHECK(read_any(p, h, d, w) == CKPT_OK);
    CHECK(d == d0 && w == w0 && std::memcmp(&h, &good, sizeof h) == 0);
    const std::vector<unsigned char> file = slurp(p);
    // every truncation, and trailing data
    for (size_t n = 0; n < file.size(); ++n) {
        spit(p, std::vector<unsigned char>(file.begin(), file.begin() + n));
        CHECK(read_any(p, h, d, w) != CKPT_OK);
    }
    std::vector<unsigned char> longer = file;
    longer.push_back(0);
    spit(p, longer);
    CHECK(read_any(p, h, d, w) != CKPT_OK);
    // random corruptions: 1..8 bytes overwritten anywhere
    for (int it = 0; it < 20000; ++it) {
        std::vector<unsigned char> bad = file;
        const int nb = 1 + (int)(rng() % 8);
        bool changed = false;
        for (int k = 0; k < nb; ++k) {
            const size_t at = (size_t)(rng() % bad.size());
            const unsigned char v = (unsigned char)rng();
            changed |= bad[at] != v;
            bad[at] = v;
        }
        spit(p, bad);
        const ckpt_status s = read_any(p, h, d, w);
        if (changed) CHECK(s != CKPT_OK);
    }
    // header-only corruptions of the same size with a recomputed checksum:
    // a header that passes the checks must describe exactly this file
    for (int it = 0; it < 20000; ++it) {
        H bad = good;
        unsigned char* b = reinterpret_cast<unsigned char*>(&bad);
        const int nb = 1 + (int)(rng() % 4);
        for (int k = 0; k < nb; ++k) b[rng() % sizeof bad] = (unsigned char)rng();
        write_with_checksum(p, bad, nd, nw);
        const ckpt_status s = read_any(p, h, d, w);
        CHECK(s == CKPT_OK || s == CKPT_BAD_HEADER || s == CKPT_BAD_SIZE);
        if (s == CKPT_OK) CHECK(d.size() == nd && w.size() == nw);
    }
}

int main() {
    std::mt19937_64 rng(20261203);
    const std::string dir = std::getenv("FUZZ_DIR") ? std::getenv("FUZZ_DIR") : "/tmp";
    const std::string p = dir + "/fuzz_ckpt.bin";

    // SU(3) 4x4x2x2, MRG32k3a states
    su_header su;
    su_header_init(su);
    su.group = 3;
    su.dims[0] = 4;
    su.dims[1] = 4;
    su.dims[2] = 2;
    su.dims[3] = 2;
    su.storage = 0;
    su.rng = 0;
    su.start = 1;
    su.nhit = 10;
    su.beta = 5.7;
    su.rng_const = 0.5;
    su.seed = 7;
    su.n_doubles = 64 * 4 * 18;
    su.n_mrg = 64 * 6;
    CHECK(su_header_valid(su));
    fuzz_file(p, su, su.n_doubles, su.n_mrg, rng);

    // crafted SU(N) headers with consistent checksums and huge sizes: the
    // reader must refuse them before allocating anything
    {
        su_header h = su;
        h.dims[0] = h.dims[1] = h.dims[2] = h.dims[3] = 65536;  // V = 2^64 wraps to 0
        h.n_doubles = 0;
        h.n_mrg = 0;
        CHECK(!su_header_valid(h));
        write_with_checksum(p, h, 0, 0);
        su_header r;
        std::vector<double> d;
        std::vector<uint32_t> w;
        CHECK(read_su_checkpoint(p.c_str(), r, d, w) == CKPT_BAD_HEADER);
        h.dims[0] = h.dims[1] = h.dims[2] = 1024;  // consistent but enormous
        h.dims[3] = 1024;
        h.n_doubles = (uint64_t)1 << 42;
        CHECK(!su_header_valid(h));
        h.dims[0] = 512;
        h.dims[1] = h.dims[2] = 256;
        h.dims[3] = 64;  // 2^31 sites: a valid geometry whose payload the file lacks
        h.n_doubles = ((uint64_t)1 << 31) * 72;
        h.n_mrg = ((uint64_t)1 << 31) * 6;
        CHECK(su_header_valid(h));
        write_with_checksum(p, h, 0, 0);
        CHECK(read_su_checkpoint(p.c_str(), r, d, w) == CKPT_BAD_SIZE);
        h = su;
        h.beta = -1.0;
        CHECK(!su_header_valid(h));
        h.beta = std::nan("");
        CHECK(!su_header_valid(h));
        h = su;
        h.dims[2] = 3;
        CHECK(!su_header_valid(h));
        h = su;
        h.group = 2;
        h.storage = 2;
        CHECK(!su_header_valid(h));
    }
    {
        su_header r;
        std::vector<double> d;
        std::vector<uint32_t> w;
        CHECK(read_su_checkpoint((dir + "/does_not_exist.bin").c_str(), r, d, w) == CKPT_CANNOT_OPEN);
    }

    // O(4) 4x2x2x2, RANLUX states
    on_header on;
    on_header_init(on);
    on.ncomp = 4;
    on.dims[0] = 4;
    on.dims[1] = on.dims[2] = on.dims[3] = 2;
    on.storage = 1;
    on.rng = 3;
    on.start = 1;
    on.nhit = 100;
    on.kappa = 0.3;
    on.lambda = 1.0;
    on.delta = 0.55;
    on.n_doubles = 32 * 4;
    on.n_words = 32 * 25;
    CHECK(on_header_valid(on));
    fuzz_file(p, on, on.n_doubles, on.n_words, rng);

    // tuning cache: round trip, then arbitrary text
    std::map<std::string, std::vector<int>> m = {{"passkinds_s0_3_32_32_32_8_gfx950", {128, 0, 1, 0, 0, 0, 0, 0, 256, 4, -1, 8, 4, 4, 2, 1}},
                                                 {"batch_s1_64_12345_gfx950", {128, 2, 0}}};
    CHECK(parse_tune_cache(format_tune_cache(m)) == m);
    const std::string text = format_tune_cache(m);
    for (size_t n = 0; n <= text.size(); ++n) (void)parse_tune_cache(text.substr(0, n));
    const char alphabet[] = "{}[]\",:-0123456789 \nabc";
    for (int it = 0; it < 50000; ++it) {
        std::string t;
        const int len = (int)(rng() % 200);
        for (int k = 0; k < len; ++k) t += (rng() % 4) ? alphabet[rng() % (sizeof alphabet - 1)] : (char)rng();
        (void)parse_tune_cache(t);
    }
    CHECK(parse_tune_cache("{\"k\": [99999999999999999999, -5, 3]}")["k"] == std::vector<int>({-5, 3}));
    CHECK(parse_tune_cache("{\"k\": [1, 2").empty());

    std::remove(p.c_str());
    if (failures) {
        std::fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    std::printf("host I/O fuzzing: ok\n");
    return 0;
}
