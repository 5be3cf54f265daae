// Host-only file formats (see lat_hostio.hpp).
#include "lat_hostio.hpp"

#include <cerrno>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>

namespace lathost {

namespace {

const char SU_MAGIC[8] = {'L', 'A', 'T', 'C', 'K', 'P', 'T', '1'};
const char ON_MAGIC[8] = {'L', 'A', 'T', 'O', 'N', 'C', 'K', '1'};

// Extents even, in [2, 2^16]; the half lattice below 2^31 sites.  *V gets
// the number of sites.
bool extents_ok(const uint32_t d[4], uint64_t* V) {
    uint64_t v = 1;
    for (int k = 0; k < 4; ++k) {
        if (d[k] < 2 || d[k] > 65536 || (d[k] & 1)) return false;
        v *= d[k];  // v <= 2^32 before the product and d <= 2^16: no overflow
        if (v / 2 > 0x7FFFFFFFull) return false;
    }
    *V = v;
    return true;
}

int state_words(uint32_t rng) { return rng == 0 ? 6 : rng == 3 ? 25 : 0; }  // MRG32k3a, RANLUX

long file_size(FILE* f) {
    if (std::fseek(f, 0, SEEK_END) != 0) return -1;
    const long n = std::ftell(f);
    if (std::fseek(f, 0, SEEK_SET) != 0) return -1;
    return n;
}

template <class H>
ckpt_status read_any(const char* path, H& h, bool (*valid)(const H&), uint64_t H::*n_doubles,
                     uint64_t H::*n_words, std::vector<double>& d, std::vector<uint32_t>& w) {
    FILE* f = std::fopen(path, "rb");
    if (!f) return CKPT_CANNOT_OPEN;
    const long size = file_size(f);
    if (size < (long)sizeof(H) || std::fread(&h, sizeof h, 1, f) != 1 || !valid(h)) {
        std::fclose(f);
        return CKPT_BAD_HEADER;
    }
    const uint64_t nd = h.*n_doubles, nw = h.*n_words;
    // the header is valid, so nd and nw are bounded by the geometry (< 2^40)
    const uint64_t want = sizeof(H) + 8 * nd + 4 * nw + 8;
    if ((uint64_t)size != want) {
        std::fclose(f);
        return CKPT_BAD_SIZE;
    }
    try {
        d.assign(nd, 0.0);
        w.assign(nw, 0u);
    } catch (const std::bad_alloc&) {
        std::fclose(f);
        return CKPT_NO_MEMORY;
    }
    uint64_t stored = 0;
    bool ok = std::fread(d.data(), sizeof(double), d.size(), f) == d.size();
    if (!w.empty()) ok = ok && std::fread(w.data(), 4, w.size(), f) == w.size();
    ok = ok && std::fread(&stored, sizeof stored, 1, f) == 1;
    std::fclose(f);
    if (!ok) return CKPT_BAD_SIZE;
    uint64_t sum = 1469598103934665603ull;
    sum = fnv1a(sum, &h, sizeof h);
    sum = fnv1a(sum, d.data(), d.size() * sizeof(double));
    if (!w.empty()) sum = fnv1a(sum, w.data(), w.size() * 4);
    return sum == stored ? CKPT_OK : CKPT_BAD_CHECKSUM;
}

}  // namespace

void su_header_init(su_header& h) {
    std::memset(&h, 0, sizeof h);
    std::memcpy(h.magic, SU_MAGIC, 8);
    h.version = 2;
}

void on_header_init(on_header& h) {
    std::memset(&h, 0, sizeof h);
    std::memcpy(h.magic, ON_MAGIC, 8);
    h.version = 1;
}

bool su_header_valid(const su_header& h) {
    if (std::memcmp(h.magic, SU_MAGIC, 8) != 0 || h.version != 2) return false;
    if (h.group != 2 && h.group != 3) return false;
    if (h.storage > 3 || (h.group == 2 && h.storage >= 2)) return false;  // 12-real forms are SU(3) only
    if (h.rng > 3 || h.start > 1 || h.nhit < 1 || h.nhit > 127 || h.frozen > 1) return false;
    if (!(h.beta >= 0.0) || h.beta > 1e300) return false;  // rejects NaN
    uint64_t V = 0;
    if (!extents_ok(h.dims, &V)) return false;
    const uint64_t ncomp = h.group == 3 ? 18 : 4;
    return h.n_doubles == V * 4 * ncomp && h.n_mrg == V * (uint64_t)state_words(h.rng);
}

bool on_header_valid(const on_header& h) {
    if (std::memcmp(h.magic, ON_MAGIC, 8) != 0 || h.version != 1) return false;
    if (h.ncomp < 1 || h.ncomp > 4 || h.storage > 1 || h.rng > 3 || h.start > 1) return false;
    if (h.nhit < 1 || h.nhit > 1000) return false;
    uint64_t V = 0;
    if (!extents_ok(h.dims, &V)) return false;
    return h.n_doubles == V * h.ncomp && h.n_words == V * (uint64_t)state_words(h.rng);
}

uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
    const unsigned char* c = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) {
        h ^= c[i];
        h *= 1099511628211ull;
    }
    return h;
}

bool write_checkpoint(const char* path, const void* header, size_t header_bytes, const double* d, size_t nd,
                      const uint32_t* w, size_t nw) {
    uint64_t sum = 1469598103934665603ull;
    sum = fnv1a(sum, header, header_bytes);
    if (nd) sum = fnv1a(sum, d, nd * sizeof(double));
    if (nw) sum = fnv1a(sum, w, nw * 4);
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return false;
    bool ok = std::fwrite(header, header_bytes, 1, f) == 1;
    if (nd) ok = ok && std::fwrite(d, sizeof(double), nd, f) == nd;
    if (nw) ok = ok && std::fwrite(w, 4, nw, f) == nw;
    ok = ok && std::fwrite(&sum, sizeof sum, 1, f) == 1;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return false;
    }
    return true;
}

ckpt_status read_su_checkpoint(const char* path, su_header& h, std::vector<double>& d, std::vector<uint32_t>& w) {
    return read_any<su_header>(path, h, su_header_valid, &su_header::n_doubles, &su_header::n_mrg, d, w);
}

ckpt_status read_on_checkpoint(const char* path, on_header& h, std::vector<double>& d, std::vector<uint32_t>& w) {
    return read_any<on_header>(path, h, on_header_valid, &on_header::n_doubles, &on_header::n_words, d, w);
}

std::map<std::string, std::vector<int>> parse_tune_cache(const std::string& t) {
    std::map<std::string, std::vector<int>> m;
    size_t i = 0;
    while (i < t.size()) {
        const size_t k0 = t.find('"', i);
        if (k0 == std::string::npos) break;
        const size_t k1 = t.find('"', k0 + 1);
        if (k1 == std::string::npos) break;
        const size_t lb = t.find('[', k1), rb = t.find(']', k1);
        if (lb == std::string::npos || rb == std::string::npos || rb < lb) break;
        std::vector<int> v;
        // the numbers between the brackets; anything else there is skipped
        size_t c = lb + 1;
        while (c < rb) {
            const char ch = t[c];
            if ((ch >= '0' && ch <= '9') || ch == '-') {
                size_t e = c + 1;
                while (e < rb && t[e] >= '0' && t[e] <= '9') ++e;
                const std::string num = t.substr(c, e - c);
                errno = 0;
                char* end = nullptr;
                const long x = std::strtol(num.c_str(), &end, 10);
                if (end != num.c_str() && errno == 0 && x >= INT_MIN && x <= INT_MAX) v.push_back((int)x);
                c = e;
            } else {
                ++c;
            }
        }
        m[t.substr(k0 + 1, k1 - k0 - 1)] = v;
        i = rb + 1;
    }
    return m;
}

std::string format_tune_cache(const std::map<std::string, std::vector<int>>& m) {
    std::string out = "{";
    bool first = true;
    for (const auto& kv : m) {
        out += first ? "\n  \"" : ",\n  \"";
        out += kv.first + "\": [";
        for (size_t j = 0; j < kv.second.size(); ++j) out += (j ? ", " : "") + std::to_string(kv.second[j]);
        out += "]";
        first = false;
    }
    return out + "\n}\n";
}

}  // namespace lathost
