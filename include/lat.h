/*
 * lat.h - C ABI of the MI355X lattice gauge Monte Carlo library (liblat.so).
 *
 * The library runs the checkerboard (even/odd) Wilson-action link sweep for
 * SU(2) and SU(3) gauge fields on one AMD Instinct MI355X (gfx950): staple
 * sum, SU(2) heat bath (Cabibbo-Marinari subgroups for SU(3)),
 * overrelaxation, reunitarisation, per-site random streams, and the
 * plaquette / Polyakov-loop reductions.  The problem statement follows the
 * QCDGPU paper (arXiv:1310.7087): SU(N) gluodynamics in an external
 * (chromo)magnetic field at finite temperature (abstract, Sec. 1 and 6);
 * lattice geometry, gauge group and precision as build-time choices and the
 * coupling and "magnetic field flux" as run-time parameters (Sec. 3.2);
 * checkerboard (pseudo-)heat bath (Sec. 3.3); selectable generator with one
 * seed parameter, 0 meaning "system time" (Sec. 3.4); hot start, NHIT = 10
 * tries and reunitarisation (Sec. 5); periodic state saving (Sec. 3.1).
 * The lat_on_* calls at the end run the paper's second model family, O(N)
 * models (N-vector fields on the sites, Metropolis update, Sec. 3.3 and 5).
 *
 * Conventions shared by every call:
 *   - Extents Nx, Ny, Nz, Nt are even and >= 2 (the checkerboard with
 *     periodic boundaries requires even extents); mu = 0,1,2,3 = x,y,z,t.
 *   - Canonical host link format ("W-frame"): FP64, site-major,
 *     site i = x + Nx*(y + Ny*(z + Nz*t)), then mu, then components:
 *       SU(3): 18 doubles, row-major 3x3, (re, im) interleaved;
 *       SU(2): 4 doubles, quaternion (a0,a1,a2,a3) = a0 1 + i(a1 s1 + a2 s2 + a3 s3).
 *     W = U * B contains the fixed background B of the flux (see lat_create).
 *   - Every call returns an int status (LAT_OK = 0, negative on error);
 *     lat_last_error() gives a message for the calling thread.
 *   - A handle is not thread-safe; different handles may be used from
 *     different threads.
 *   - Work is queued on the handle's HIP stream: lat_sweep and lat_run (and
 *     the batch equivalents) are asynchronous; lat_measure, lat_get_*,
 *     lat_set_links and lat_save synchronise that stream.
 */
#ifndef LAT_H
#define LAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define LAT_OK 0
#define LAT_EINVAL (-1)       /* bad argument: odd/too small extent, group not 2|3,
                                 beta < 0 or NaN, NULL output, wrong buffer size */
#define LAT_ENOMEM (-2)       /* device or host allocation failed, or caller buffer too small */
#define LAT_EDEVICE (-3)      /* a HIP call failed; the message names it */
#define LAT_EIO (-4)          /* checkpoint file could not be read or written */
#define LAT_ECORRUPT (-5)     /* checkpoint checksum or header mismatch */
#define LAT_ESTATE (-6)       /* call not valid in the handle's current state */
#define LAT_EUNSUPPORTED (-7) /* combination not supported (e.g. 12-real SU(2)) */

/* ---- link storage forms ---- */
#define LAT_F64 0      /* FP64, all reals stored (18 for SU(3), 4 for SU(2)) */
#define LAT_F32 1      /* FP32 storage and staple/subgroup arithmetic; FP64 for
                          reunitarisation, heat-bath acceptance and observable sums */
#define LAT_F32_C12 2  /* as LAT_F32, SU(3) only: first two rows stored (12 reals),
                          row 3 = conj(row1 x row2) rebuilt on every load */
#define LAT_F64_C12 3  /* FP64 arithmetic, SU(3) only: first two rows stored
                          (12 doubles), row 3 = conj(row1 x row2) rebuilt in FP64
                          on every load; two thirds of LAT_F64's link bytes */

/* ---- random number generators (one parameter picks it, Sec. 3.4) ---- */
#define LAT_RNG_MRG32K3A 0  /* per-site MRG32k3a streams, 2^127 apart */
#define LAT_RNG_PHILOX 1    /* per-site counter-based Philox4x32-10 */
#define LAT_RNG_CONST 2     /* every uniform = rng_const (debugging, Sec. 3.4); an
                               SU(3) hot start with it is refused (LAT_EINVAL): equal
                               uniforms give two equal Gaussian rows */
#define LAT_RNG_RANLUX 3    /* per-site RANLUX, luxury level 3 (the generator of the
                               paper's benchmark runs, Sec. 5): of every 223 outputs
                               of the subtract-with-borrow generator x_n = x_{n-10}
                               - x_{n-24} - c mod 2^24 the first 24 are used; site i
                               is seeded with 1 + (seed + 1000003 (i + 2654435761
                               lattice_id)) mod 2147483561 by the standard
                               40014-multiplier procedure; each link update begins
                               a new block of 24 */

#define LAT_FROZEN_NONE 0  /* every link is updated */
#define LAT_FROZEN_T0 1    /* spatial links at t = 0 held at the background */

#define LAT_COLD 0  /* unit links */
#define LAT_HOT 1   /* Haar-random links */

typedef struct lat_ctx* lat_t;
typedef struct lat_batch* lat_batch_t;

typedef struct {
    int storage;         /* LAT_F64 (default), LAT_F32, LAT_F32_C12, LAT_F64_C12 */
    int rng;             /* LAT_RNG_PHILOX (default), LAT_RNG_MRG32K3A, LAT_RNG_CONST,
                            LAT_RNG_RANLUX */
    double rng_const;    /* value of every uniform for LAT_RNG_CONST, in (0,1) */
    int start;           /* LAT_HOT (default) or LAT_COLD */
    uint64_t seed;       /* run seed; 0 = derived from the system time and reported
                            by lat_get_info. MRG32k3a needs 1 <= seed < 4294944443. */
    int nhit;            /* heat-bath tries per SU(2) (sub)update, 1..127; default 10 */
    uint32_t lattice_id; /* second Philox counter word: distinguishes lattices
                            that share a seed */
    void* stream;        /* hipStream_t to queue work on (e.g. torch's current
                            stream); NULL = a stream the library creates */
    void* device_buffer; /* optional caller-owned device memory for all device
                            state; it must stay alive until lat_destroy */
    size_t device_bytes; /* its size; see lat_device_bytes */
    int block_size;      /* work-group size of the sweep kernels: 0 = tuned
                            default, else 64, 128 or 256 */
    int tile_order;      /* work-group -> tile map: 0 = one z-slab per XCD (own
                            L2) when 8 | Nz, else identity (default); 1 = identity;
                            2 = reversed (order-independence tests);
                            3 = one contiguous range of tiles per XCD;
                            4 = with a 4-D tile only: one z-slab of tiles per
                            XCD, tiles walked x, y, t, then z */
    int layout;          /* plane stride of the link arrays: 0 = staggered so that
                            planes do not alias in caches and channels (default),
                            1 = plain (padded to a multiple of 256 sites) */
    int tile[4];         /* sites of one parity per work-group as a 4-D tile
                            (x/2, y, z, t), product 64, 128 or 256; all 0 =
                            runs of block_size consecutive sites (default) */
    int max_waves_per_simd; /* occupancy cap of the sweep kernels: 0 = default for
                            the form (1 for SU(3) FP64, whose staple traffic then
                            fits the L2 better; none otherwise), -1 = none, 1..8 */
    int frozen;          /* LAT_FROZEN_NONE (default) or LAT_FROZEN_T0: the
                            spatial links of the time slice t = 0 are set to the
                            background field (U = 1, W = B) and never updated, so
                            that the external field (Sec. 1, Sec. 3.2 "field
                            flux") can no longer be removed by a change of
                            variables; no random numbers are drawn for them */
    int stage_lds;       /* SU(3) with a 4-D tile (see tile) whose extents divide
                            the lattice, not RANLUX: 1 = each work-group first
                            copies the opposite-parity U_mu links its sites read
                            (six reads per link) into LDS and takes them from
                            there; 0 = every link read goes through the caches
                            (default).  Results are identical. */
} lat_options;

/* Fills *opt with the defaults listed above. */
void lat_default_options(lat_options* opt);

/* Device bytes a lattice with these parameters needs (links, generator
 * state, reduction scratch).  Returns 0 for invalid parameters. */
size_t lat_device_bytes(int group, int Nx, int Ny, int Nz, int Nt, const lat_options* opt);

/*
 * Creates one lattice on the current HIP device and initialises it (cold or
 * Haar-random links, times the background B).
 *   group: 2 or 3 (SU(N)); beta: Wilson coupling >= 0.
 *   field_flux: integer number n of flux quanta of a constant Abelian
 *     chromomagnetic background along lambda_3 (T = diag(1,-1[,0])) through
 *     the x-y planes: phi = 2 pi n / (Nx Ny) per x-y plaquette, realised by
 *     the fixed links B_y(x) = exp(i phi x T) and, at x = Nx-1,
 *     B_x(x) = exp(-i phi Nx y T).  The stored links are W = U B.
 *   opt: NULL for defaults.  On success *out is a new handle.
 */
int lat_create(lat_t* out, int group, int Nx, int Ny, int Nz, int Nt, double beta,
               int field_flux, const lat_options* opt);

/*
 * One compound sweep (asynchronous): n_hb heat-bath sweeps, then n_or
 * overrelaxation sweeps.  Each sweep is 8 dependent checkerboard passes
 * (mu = 0..3, parity 0 then 1).  Every link is reunitarised (in FP64) right
 * after its last update of the compound sweep.  n_hb, n_or >= 0.
 */
int lat_sweep(lat_t h, int n_hb, int n_or);

/*
 * n_sweeps compound sweeps with a measurement after every measure_every-th
 * one (0 = none), all queued without host synchronisation; the series are
 * copied to the host at the end (this call synchronises).
 *   plaq_series: [k][3] (P, P_s, P_t) or NULL; poly_series: [k][2] or NULL,
 *   k = n_sweeps / measure_every measurements.
 */
int lat_run(lat_t h, int n_sweeps, int n_hb, int n_or, int measure_every,
            double* plaq_series, double* poly_series);

/*
 * Measures (synchronously) the average plaquette
 *   plaq[0] = P = (P_s + P_t)/2, plaq[1] = P_s (3 spatial planes),
 *   plaq[2] = P_t (3 planes with t), each (1/N) Re Tr of
 *   W_mu(x) W_nu(x+mu) W_mu(x+nu)^+ W_nu(x)^+,
 * and the Polyakov loop poly = (Re, Im) of the spatial average of
 *   (1/N) Tr prod_{t=0}^{Nt-1} W_t(x, t).
 * Sums are FP64 with a compensated final reduction in a fixed order.
 */
int lat_measure(lat_t h, double plaq[3], double poly[2]);

/* Canonical FP64 links (see top); n_doubles must equal 4*V*ncomp. */
int lat_get_links(lat_t h, double* host, size_t n_doubles);
/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture elsewhere in the process, tight serving loops, harnesses that
 * forbid hipMalloc): the same canonical FP64 links as lat_get_links, bit for
 * bit, without any device or host allocation.  The links pass through one
 * fixed device array of LAT_NOALLOC_SCRATCH_BYTES per GPU, which the library
 * holds from the first call on that GPU until the process ends, in chunks
 * of whole sites (so every lattice size is accepted; no chunk exceeds the
 * array).  n_doubles must equal 4*V*ncomp (LAT_EINVAL otherwise).
 * Synchronises the handle's stream.  Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (other threads, other handles) race
 * and must be serialised by the caller.
 */
#define LAT_NOALLOC_SCRATCH_BYTES (16u << 20)
int lat_get_links_noalloc(lat_t h, double* host, size_t n_doubles);
/* Replaces all links (rounded to the storage form; 12-real keeps rows 1-2). */
int lat_set_links(lat_t h, const double* host, size_t n_doubles);
/* Per-site generator states in canonical site order: MRG32k3a 6 words per
 * site (x1[n-3], x1[n-2], x1[n-1], x2[n-3], x2[n-2], x2[n-1]); RANLUX 25
 * words per site (the last delivered block of 24 subtract-with-borrow
 * outputs, oldest first, then carry | 2 while no block has been delivered);
 * n_words = words * V.  LAT_ESTATE for the stateless generators. */
int lat_get_rng_state(lat_t h, uint32_t* host, size_t n_words);
/*
 * Kernel profiling (the paper's run-time kernel profiling, Sec. 3.2): runs
 * `reps` compound sweeps (n_hb, n_or) with the passes launched directly on
 * the handle's stream, HIP events before the heat-bath passes, between the
 * two kinds and after the overrelaxation passes, and returns the average
 * duration in milliseconds of a heat-bath pass (ms_hb) and of an
 * overrelaxation pass (ms_or), each the span of its back-to-back passes
 * divided by their number.  The lattice advances as with lat_sweep.
 * Synchronises.  Either output may be NULL.
 */
int lat_profile_passes(lat_t h, int n_hb, int n_or, int reps, double* ms_hb, double* ms_or);

/*
 * Autotuner (the paper foresees auto-tuning of launch parameters from
 * profiling, Sec. 6): heat-bath and overrelaxation passes get launch shapes
 * of their own.  For each kind that the compound sweep (n_hb, n_or) runs,
 * every candidate -- work-group size (64, 128, 256) x work-group order (0, 1)
 * x occupancy cap (none, 1, 2, 3 waves per SIMD), and for SU(3) the
 * LDS-staged 4-D tiles (8,4,4,2), (8,2,4,4), (4,2,4,4), (4,4,2,4) that
 * divide the lattice (see stage_lds) -- is timed on sweeps of that kind from
 * the same saved device state; the fastest is kept, and the lattice's device
 * state and counters are restored, so the Markov chain is unchanged (results
 * do not depend on the shape).  If the environment variable LAT_TUNE_CACHE
 * names a file, choices are read from and added to it: a JSON object mapping
 * a key (storage, group, extents, device) to both kinds' shapes (16 integers,
 * as lat_get_launch_shape gives them), rewritten atomically.  result
 * (optional) receives {work-group size, order, cap (-1 = none)} of the
 * overrelaxation shape (of the heat-bath shape if n_or = 0).  Synchronises.
 * LAT_ESTATE with the accept log on or an explicit 4-D tile.
 */
int lat_autotune(lat_t h, int n_hb, int n_or, int result[3]);
/* Launch shape of the heat-bath (kind 0) or overrelaxation (kind 1) passes:
 * {work-group size, order, cap (-1 = none), tile x/2, y, z, t (0 = runs of
 * consecutive sites), LDS-staged (0/1)}. */
int lat_get_launch_shape(lat_t h, int kind, int shape[8]);

/* Any output pointer may be NULL. */
int lat_get_info(lat_t h, uint64_t* seed_used, uint64_t* hb_sweeps_done, uint64_t* sweeps_done);

/*
 * Heat-bath accept log (debugging): when on, the next compound sweeps record
 * for every heat-bath update the accepted try index (or -1 if all NHIT tries
 * were rejected or the update was skipped), one int8 per
 * [hb sweep k of the last compound sweep][mu][canonical site][subgroup g < 3].
 * lat_get_accept_log copies min(n, available) bytes and returns that count
 * (>= 0) or a negative status.
 */
int lat_set_accept_log(lat_t h, int on);
int64_t lat_get_accept_log(lat_t h, int8_t* host, size_t n);

/*
 * Portable checkpoint (little-endian, checksummed): parameters, counters,
 * canonical FP64 W-frame links and MRG32k3a states.  lat_load creates a new
 * handle (storage and stream from opt, or the saved storage if opt is NULL)
 * that continues the saved run exactly.
 */
int lat_save(lat_t h, const char* path);
int lat_load(lat_t* out, const char* path, const lat_options* opt);

/* Releases the handle; NULL is a no-op. */
int lat_destroy(lat_t h);

/* Message of the last failing call on this thread ("" if none). */
const char* lat_last_error(void);

/* Raw device Philox4x32-10 for generator checks: out[4k..4k+3] =
 * Philox4x32-10(counter ctr[4k..4k+3], key); host arrays, n blocks. */
int lat_philox4x32_10(const uint32_t* ctr, const uint32_t key[2], uint32_t* out, size_t n);

/* ------------------------------------------------------------------ */
/* Batches: many independent lattices (a parameter scan, the paper's   */
/* "trivial parallelisation", Sec. 5 and 6) advanced together: each    */
/* checkerboard pass of every member is one kernel launch covering all */
/* members, and a compound sweep is replayed as one captured graph.    */
/* ------------------------------------------------------------------ */
typedef struct {
    int group, Nx, Ny, Nz, Nt;
    double beta;
    int field_flux;
    uint64_t seed;
    int start;
    uint32_t lattice_id;
} lat_desc;

/* n lattices described by d[0..n-1]; common supplies storage, nhit, stream
 * and block_size (0 = tuned by lat_batch_autotune or the default); the
 * generator must be Philox (each member keyed by its own seed and
 * lattice_id); with LAT_F32_C12 (LAT_F64_C12) the SU(2) members use
 * LAT_F32 (LAT_F64); frozen links are not supported in a batch
 * (LAT_EUNSUPPORTED); the per-lattice fields of common are ignored.  Each member's
 * results are bit-identical to the same lattice run alone. */
int lat_batch_create(lat_batch_t* out, int n, const lat_desc* d, const lat_options* common);
/* Launch form and shape.  mode 0 (default): one kernel per pass index, each
 * covering that pass of every member (kernel boundaries order the passes),
 * every member whole on one XCD; mode 2: the same with the members' tiles
 * dealt round the XCDs (see lat_batch_autotune);
 * mode 1, a persistent work-list kernel for all passes with per-member
 * dependency counters, is switched off and returns LAT_EUNSUPPORTED.
 * block_size 64|128|256, sites_per_thread 1..8 per work item, grid = blocks
 * of the persistent kernel (0 = 1024 threads per compute unit).  Every form
 * and shape gives bit-identical results. */
int lat_batch_configure(lat_batch_t b, int mode, int block_size, int sites_per_thread, int grid);
/* Autotuner of the batch launch: times every work-group size (64, 128,
 * 256) x sites per thread (1, 2, 4) x XCD map -- 0: every member whole on
 * one XCD (members packed largest first onto the XCD with the least work,
 * so a member's neighbour links stay in one L2; the default), 1: the
 * members' tiles dealt round the XCDs (a member larger than one L2 spreads
 * over all of them) -- on compound sweeps (n_hb, n_or) of the whole batch,
 * keeps the fastest and restores every member's state (cache file as for
 * lat_autotune).  result (optional) = {size, sites per thread}.
 * Synchronises. */
int lat_batch_autotune(lat_batch_t b, int n_hb, int n_or, int result[2]);
/* Current batch launch shape: {work-group size, sites per thread, XCD map}. */
int lat_batch_get_shape(lat_batch_t b, int shape[3]);
/* n_sweeps compound sweeps of every member; if plaq / poly are non-NULL they
 * receive each member's final measurement ([n][3] and [n][2]); synchronises. */
int lat_batch_run(lat_batch_t b, int n_sweeps, int n_hb, int n_or, double* plaq, double* poly);
int lat_batch_get_links(lat_batch_t b, int i, double* host, size_t n_doubles);
int lat_batch_set_links(lat_batch_t b, int i, const double* host, size_t n_doubles);
int lat_batch_destroy(lat_batch_t b);

/* ------------------------------------------------------------------ */
/* O(N) models (the paper's second model family, Sec. 3.3 and 5): an   */
/* N-vector field phi(x) on the sites, N = 1..4, with the lattice       */
/* phi^4 action in hopping-parameter form and a constant source h      */
/* along component 0 (the external field):                             */
/*   S = sum_x [ -2 kappa sum_mu phi(x).phi(x+mu) + phi(x)^2            */
/*               + lambda (phi(x)^2 - 1)^2 - h phi_0(x) ].              */
/* The paper names the model, its coupling-constant dependence (Sec. 1) */
/* and an improved Metropolis update with NHIT = 100 tries per site     */
/* (Sec. 3.3, Sec. 5) but writes out neither; this form is the reading. */
/* ------------------------------------------------------------------ */
typedef struct lat_on_ctx* lat_on_t;

/* Device bytes of an O(N) field with these parameters (0 if invalid). */
size_t lat_on_device_bytes(int ncomp, int Nx, int Ny, int Nz, int Nt, const lat_options* opt);

/*
 * Creates an O(N) field on the current HIP device and initialises it: cold
 * phi = (1, 0, ..), hot phi_a = 2 u_a - 1 (uniform in the cube [-1, 1]^N).
 *   ncomp: N in 1..4; kappa: hopping parameter (finite); lambda >= 0;
 *   h: source along component 0; delta > 0: proposal half-width.
 *   opt: storage LAT_F64 or LAT_F32 (field storage; all update and
 *   reduction arithmetic is FP64 in both), rng any of the four generators
 *   (MRG32k3a: 1 <= seed < 4294944443, else LAT_EINVAL), nhit = hits
 *   per site and sweep 1..1000 (NULL opt: 100, the paper's value), seed,
 *   lattice_id, start, stream, device_buffer/device_bytes and block_size as
 *   for lat_create; frozen must be LAT_FROZEN_NONE; the tile, layout and
 *   occupancy fields are ignored.
 * Draws: Philox counter (canonical site, lattice_id, sweep number, hit k)
 * gives one 4-word block per hit: u_a from the high 24 bits of word a
 * (a < N), the acceptance uniform from the low bytes of words 0, 1, 2; the
 * hot start uses counter (site, lattice_id, 0, 0xFFFFFFFF).  RANLUX (seeded
 * as for lat_create): every site update begins a new block, each hit takes
 * N values then the acceptance value; the hot start takes the first N values
 * of the first block.  MRG32k3a (site streams 2^127 apart, as for
 * lat_create): drawn in sequence, the hot start N values, each hit N values
 * then the acceptance value.
 */
int lat_on_create(lat_on_t* out, int ncomp, int Nx, int Ny, int Nz, int Nt, double kappa, double lambda,
                  double h, double delta, const lat_options* opt);

/*
 * n_sweeps sweeps (asynchronous).  A sweep updates every site of parity 0,
 * then every site of parity 1 (the neighbours of a site have the other
 * parity); each site gets NHIT successive Metropolis hits with its
 * neighbours fixed: phi' = phi + delta (2u - 1), accepted iff
 * u_acc < exp(-(s(phi') - s(phi))) with the local action
 * s(phi) = -2 kappa F.phi + phi.phi + lambda (phi.phi - 1)^2 - h phi_0,
 * F = sum_mu [phi(x+mu) + phi(x-mu)].
 */
int lat_on_sweep(lat_on_t h, int n_sweeps);

/*
 * Measures (synchronously) obs = { <phi^2>, <phi(x).phi(x+mu)> averaged
 * over sites and the 4 directions, <(phi^2 - 1)^2>, <phi_0>, <phi_1>,
 * <phi_2>, <phi_3> } (components beyond N are 0).  FP64 sums in a fixed
 * order with a compensated final reduction.  The action per site is
 * -8 kappa obs[1] + obs[0] + lambda obs[2] - h obs[3].
 */
int lat_on_measure(lat_on_t h, double obs[7]);

/* n_sweeps sweeps with a measurement after every measure_every-th (0 =
 * none) into series[k][7] (may be NULL), k = n_sweeps / measure_every;
 * synchronises at the end. */
int lat_on_run(lat_on_t h, int n_sweeps, int measure_every, double* series);

/* Accepted hits of the most recent sweep / (V * NHIT); synchronises.
 * LAT_ESTATE before the first sweep. */
int lat_on_acceptance(lat_on_t h, double* rate);

/* Field as FP64 [site i][component a], i canonical; n_doubles = V * N.
 * set rounds to the storage form.  Both synchronise. */
int lat_on_get_field(lat_on_t h, double* host, size_t n_doubles);
int lat_on_set_field(lat_on_t h, const double* host, size_t n_doubles);
int lat_on_get_info(lat_on_t h, uint64_t* seed_used, uint64_t* sweeps_done);

/* Runs `reps` sweeps launched back to back between two HIP events on the
 * handle's stream and returns the average duration of one pass (half a
 * sweep) in milliseconds.  The field advances as with lat_on_sweep. */
int lat_on_profile(lat_on_t h, int reps, double* ms_per_pass);

/*
 * Portable checkpoint of an O(N) field (the paper's periodic state saving,
 * Sec. 3.1; little-endian, FNV-1a checksummed): parameters, sweep counter,
 * the canonical FP64 field and, for RANLUX and MRG32k3a, every site's
 * generator state.
 * lat_on_load creates a new handle (storage, stream and device buffer from
 * opt, or the saved storage if opt is NULL; generator, seed, NHIT and
 * lattice id always from the file) that continues the saved chain exactly.
 * LAT_EIO if the file cannot be read or written, LAT_ECORRUPT on a bad
 * header, size or checksum.
 */
int lat_on_save(lat_on_t h, const char* path);
int lat_on_load(lat_on_t* out, const char* path, const lat_options* opt);

/* Releases the handle; NULL is a no-op. */
int lat_on_destroy(lat_on_t h);

#ifdef __cplusplus
}
#endif
#endif /* LAT_H */
