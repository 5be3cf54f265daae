// Host-only file formats of the library: the portable checkpoints of SU(N)
// lattices and O(N) fields (the paper's periodic state saving, Sec. 3.1) and
// the launch-shape tuning cache.  Plain C++ with no HIP dependence, so that
// the parsers can be built and fuzzed on their own.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <map>
#include <string>
#include <vector>

namespace lathost {

// Status of a checkpoint read.
enum ckpt_status { CKPT_OK = 0, CKPT_CANNOT_OPEN, CKPT_BAD_HEADER, CKPT_BAD_SIZE, CKPT_BAD_CHECKSUM, CKPT_NO_MEMORY };

// SU(N) lattice checkpoint, version 2: this header (little-endian, no
// padding), then n_doubles canonical FP64 W-frame links, then n_mrg 32-bit
// generator-state words, then the FNV-1a 64 checksum of all of it.
struct su_header {
    char magic[8];  // "LATCKPT1"
    uint32_t version, group, dims[4], storage, rng, start, nhit;
    int32_t flux;
    uint32_t lat_id, frozen, reserved;
    double beta, rng_const;
    uint64_t seed, hb_sweeps, sweeps, n_doubles, n_mrg;
};
static_assert(sizeof(su_header) == 120, "SU(N) checkpoint header layout");

// O(N) field checkpoint, version 1: header, n_doubles FP64 field values
// [site][component], n_words generator-state words, checksum.
struct on_header {
    char magic[8];  // "LATONCK1"
    uint32_t version, ncomp, dims[4], storage, rng, start, nhit, lat_id, reserved;
    double kappa, lambda, h, delta, rng_const;
    uint64_t seed, sweeps, n_doubles, n_words;
};
static_assert(sizeof(on_header) == 128, "O(N) checkpoint header layout");

void su_header_init(su_header& h);
void on_header_init(on_header& h);

// Whether a header describes a checkpoint this library writes: magic and
// version, every field in its range (extents even, 2..2^16 and the half
// lattice below 2^31 sites), payload sizes that match the geometry.
bool su_header_valid(const su_header& h);
bool on_header_valid(const on_header& h);

uint64_t fnv1a(uint64_t h, const void* p, size_t n);

// Writes header, payloads and checksum to `path` (through path.tmp and a
// rename, so a failed write leaves no partial file).  false on I/O error.
bool write_checkpoint(const char* path, const void* header, size_t header_bytes, const double* d, size_t nd,
                      const uint32_t* w, size_t nw);

// Reads a checkpoint.  The header is checked first, then the file's size
// against the sizes the header announces, and only then are the payloads
// allocated and read; last the checksum.
ckpt_status read_su_checkpoint(const char* path, su_header& h, std::vector<double>& d, std::vector<uint32_t>& w);
ckpt_status read_on_checkpoint(const char* path, on_header& h, std::vector<double>& d, std::vector<uint32_t>& w);

// The tuning cache: a JSON object mapping keys to integer arrays,
// {"key": [1, 2, 3], ...}.  Only that flat form is read back; anything else
// in the text is skipped.
std::map<std::string, std::vector<int>> parse_tune_cache(const std::string& text);
std::string format_tune_cache(const std::map<std::string, std::vector<int>>& m);

}  // namespace lathost
