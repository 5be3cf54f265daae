// Plain structures shared by the host runtime and the kernels.
#pragma once
#include <stdint.h>

#define LAT_RNG_MRG_I 0
#define LAT_RNG_PHILOX_I 1
#define LAT_RNG_CONST_I 2
#define LAT_RNG_RANLUX_I 3

#define LAT_ST_F64 0
#define LAT_ST_F32 1
#define LAT_ST_F32C12 2
#define LAT_ST_F64C12 3

struct LatGeom {
    int nx, ny, nz, nt;
    int nxh;         // nx / 2
    int64_t vh;      // sites per parity
    int64_t vh_pad;  // plane length (vh rounded up)
};

// Everything one checkerboard pass needs.
struct PassArgs {
    LatGeom g;
    char* links;           // parity-split SoA link planes
    uint32_t* mrg;         // [parity][word 0..5][vh_pad] MRG32k3a states, or null
    const uint64_t* hb_count;  // device counter: heat-bath sweeps completed
    int8_t* accept_log;    // [k][mu][canonical site][3] or null
    double beta;
    double rng_const;
    uint32_t key0, key1, lat_id;
    int nhit;
    int group;
    int mu, parity;
    int hb_offset;         // index of this heat-bath sweep within the compound sweep
    int tile_order;        // 0 XCD-aware, 1 identity, 2 reversed
    int flux;
    int tshape[4];         // work-group tile (x/2, y, z, t) in sites of one parity; 0 = lexicographic runs
    int tcount[4];         // tiles per direction
    int nyb, zslab;        // z-slab order: work-groups per z-plane, z-planes per XCD
    int lds_reserve;       // dynamic LDS bytes reserved per work-group (caps occupancy)
    int reverse;           // z-slab order walked backwards (every other pass)
    int frozen;            // 1: spatial links at t = 0 are not updated
    uint64_t* bump_counter = nullptr;  // heat-bath counter the pass advances ...
    int bump_by = 0;                   // ... by this much when it is done (0: none)
    int stage_lds = 0;                 // dynamic LDS bytes of the tile's staged U_mu links (0: none)
};

// Initialisation of one lattice.
struct InitArgs {
    LatGeom g;
    char* links;
    uint32_t* mrg;
    double rng_const;
    uint32_t key0, key1, lat_id;
    int start;  // 0 cold, 1 hot
    int flux;
    int frozen;  // 1: spatial links at t = 0 start (and stay) at the background
};

// Reductions.
struct MeasArgs {
    LatGeom g;
    const char* links;
    double* partial;      // [4][nblocks]: P_s sums, P_t sums, Re L, Im L
    int nb_plaq;          // blocks of the plaquette kernel
    int nb_poly;          // blocks of the Polyakov kernel
    int nyb, zslab;       // z-slab order of the plaquette blocks (zslab 0: interleaved)
    int lds_reserve;      // dynamic LDS per plaquette work-group (caps occupancy)
};

// One member of a batch of independent lattices.
struct BatchLat {
    LatGeom g;
    char* links;
    const uint64_t* hb_count;  // heat-bath sweeps completed before this launch
    double beta;
    double rng_const;
    uint32_t key0, key1, lat_id;
    int nhit, group, flux, rng;
    int ntiles;       // tiles per pass
    int tile_prefix;  // index of this lattice's first tile within a pass
};

// One work-group's share of a batch pass: tile `tile` of member `member`
// (member < 0: nothing, the work-group leaves at once).
struct BatchItem {
    int member, tile;
};

// Work list of one persistent batch launch: n_sweeps compound sweeps
// (n_hb, n_or) of every member; item = (pass, lattice, tile), pass-major.
struct BatchArgs {
    const BatchLat* lats;
    int nlat;
    int tiles_per_pass;   // sum of ntiles over members
    int passes_per_sweep; // 8 * (n_hb + n_or)
    int n_hb, n_or, n_sweeps;
    int tile;             // half-sites per tile
    unsigned* queue;      // next work item
    unsigned* done;       // [nlat] tiles completed in this launch
    int* status;          // nonzero if a dependency wait hit its spin limit
    unsigned spin_limit;
    const BatchItem* items = nullptr;  // per-pass work-group -> (member, tile) map (one launch per pass)
    int nitems = 0;                    // work-groups of a pass launch
};
