/*
 * Plain FP64 CPU oracle for the checkerboard SU(2)/SU(3) Wilson-action
 * Monte Carlo (pseudo-heat bath, overrelaxation, reunitarisation, plaquette
 * and Polyakov loop).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The product
 * path (the HIP library under paper_1310_7087_amd/) never links, loads or
 * calls it, and shares no source, header or table with it.
 *
 * Everything is plain, unblocked FP64 in the canonical layout:
 *   site i = x + Nx*(y + Ny*(z + Nz*t)),  parity (x+y+z+t) mod 2,
 *   link (i, mu) at offset (i*4 + mu) * ncomp doubles,
 *   SU(3): 18 doubles, row-major 3x3, (re, im) interleaved;
 *   SU(2): 4 doubles, quaternion (a0,a1,a2,a3) = a0*1 + i(a1 s1 + a2 s2 + a3 s3).
 * Exported links are in the "W-frame" (dynamical link times the fixed
 * background field); internally the oracle keeps the U-frame and applies
 * the background on the fly.
 */
#ifndef LAT_ORACLE_H
#define LAT_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_lattice orc_lattice;

enum { ORC_RNG_MRG32K3A = 0, ORC_RNG_PHILOX = 1, ORC_RNG_CONST = 2, ORC_RNG_RANLUX = 3 };
enum { ORC_COLD = 0, ORC_HOT = 1 };

/* Returns NULL on invalid arguments (odd or < 2 extents, group not 2/3, an
 * SU(3) hot start with the constant generator).
 * frozen = 1 holds the spatial links of the time slice t = 0 at the
 * background field (U = 1, W = B) and never updates them: the external field
 * of the paper's Sec. 1 can then no longer be removed by a change of
 * variables (a reading: the paper names the field only as a flux). */
orc_lattice* orc_create(int group, int nx, int ny, int nz, int nt, double beta,
                        int flux, int rng, double rng_const, uint64_t seed,
                        int nhit, uint32_t lattice_id, int start, int frozen);
void orc_destroy(orc_lattice* L);
void orc_set_threads(int n);
int  orc_get_threads(void);

/* One compound sweep: n_hb heat-bath sweeps then n_or overrelaxation sweeps,
 * every sweep = mu 0..3 x parity 0,1; each link reunitarised after its last
 * update of the compound sweep. */
void orc_sweep(orc_lattice* L, int n_hb, int n_or);
/* plaq = {P, P_s, P_t}, poly = {Re L, Im L}. */
void orc_measure(const orc_lattice* L, double plaq[3], double poly[2]);
/* Canonical W-frame FP64 links, 4*V*ncomp doubles. */
void orc_get_links(const orc_lattice* L, double* out);
void orc_set_links(orc_lattice* L, const double* in);
uint64_t orc_hb_sweeps(const orc_lattice* L);
/* MRG32k3a per-site states, 6 words per site (x1[n-3],x1[n-2],x1[n-1],x2[...]). */
int  orc_get_mrg_states(const orc_lattice* L, uint32_t* out);
/* RANLUX luxury level 3 (p = 223, r = 24) raw 24-bit outputs for one seed
 * (luxury_blocks = 0: the bare subtract-with-borrow base generator). */
void orc_ranlux_raw(uint32_t seed, int n, int luxury_blocks, uint32_t* out);
/* The 10000th outputs of default-seeded ranlux24_base and ranlux24 as
 * computed by this C++ library (the standard fixes 7937952 and 9901578). */
void orc_ranlux_standard_values(uint32_t out[2]);
/* Seed of site i's RANLUX stream. */
uint32_t orc_ranlux_site_seed(uint64_t seed, int64_t i, uint32_t lattice_id);
/* Accept log of the most recent compound sweep's heat-bath updates:
 * one int8 per (hb sweep k, mu, site i, subgroup g), value = accepted try
 * index or -1.  Layout [k][mu][i][g], g < 3.  Enabled by orc_enable_accept_log. */
void orc_enable_accept_log(orc_lattice* L, int on);
int64_t orc_get_accept_log(const orc_lattice* L, int8_t* out, int64_t n);

/* ---- primitives exposed for pinning ---- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* State of site stream `site` for MRG32k3a seed s: A^(site*2^127) (s,s,s,s,s,s). */
int  orc_mrg_site_state(uint64_t seed, uint64_t site, uint32_t st[6]);
/* One MRG32k3a step; returns z in [1, m1]. */
uint32_t orc_mrg_next(uint32_t st[6]);
/* Advance a state by 2^e steps (matrix squaring), for jump checks. */
void orc_mrg_advance_pow2(uint32_t st[6], int e);
double orc_uniform24(uint32_t w);
/* Kennedy-Pendleton draw at alpha from sequential uniforms u[]
 * (4 per try, then 2 for the direction).  Returns the accepted try index or
 * -1; x[4] = (a0,a1,a2,a3) or (1,0,0,0) if rejected. *used = uniforms read. */
int  orc_kp_sample(double alpha, int nhit, const double* u, double x[4], int* used);
/* Update one link with a fixed staple: kind 0 = heat bath, 1 = overrelaxation.
 * U, Uout canonical (ncomp doubles); A is the staple as an N x N complex
 * matrix, row-major (re,im).  u[] sequential uniforms as in orc_kp_sample.
 * reunit != 0 reunitarises the result. Returns the number of uniforms read. */
int  orc_update_link(int group, double beta, int nhit, int kind, int reunit,
                     const double* U, const double* A, const double* u, double* Uout);
/* Staple of link (i, mu) in the W-frame as an N x N complex matrix. */
void orc_staple(const orc_lattice* L, int64_t i, int mu, double* A);

/* ---- O(N) phi^4 model: N-vector per site, multi-hit Metropolis ---- */
typedef struct orc_on orc_on;
/* ncomp = N in 1..4; any of the four generators; nhit 1..1000;
 * lambda >= 0, delta > 0.  Returns NULL on invalid arguments.  Field layout
 * [site i][component a], FP64. */
orc_on* orc_on_create(int ncomp, int nx, int ny, int nz, int nt, double kappa, double lambda, double h,
                      double delta, int rng, double rng_const, uint64_t seed, int nhit, uint32_t lattice_id,
                      int start);
void orc_on_destroy(orc_on* L);
void orc_on_sweep(orc_on* L, int nsweeps);
void orc_on_measure(const orc_on* L, double out[7]);
void orc_on_get_field(const orc_on* L, double* out);
void orc_on_set_field(orc_on* L, const double* in);
uint64_t orc_on_sweeps(const orc_on* L);
/* MRG32k3a states, 6 words per site; -1 for the other generators. */
int orc_on_get_mrg_states(const orc_on* L, uint32_t* out);
/* Accepted hits of the most recent sweep / (V * NHIT). */
double orc_on_acceptance(const orc_on* L);

#ifdef __cplusplus
}
#endif
#endif
