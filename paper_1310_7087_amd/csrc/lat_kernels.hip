// HIP kernels for gfx950: checkerboard heat-bath / overrelaxation passes,
// initialisation, observables and layout conversion.
//
// One thread updates one link U_mu(x) of the pass parity.  Links live in a
// parity-split structure of arrays (see lat_dev.hpp), so consecutive threads
// read consecutive 8/16-byte vectors of every plane: each of the 19 link
// reads of a staple is a fully coalesced wave-wide load, and neighbour reuse
// is served from L2 / Infinity Cache.  Work-groups are mapped so that each
// XCD (own L2) sweeps a contiguous slab of the lattice.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "lat_dev.hpp"
#include "lat_launch.hpp"

using namespace latdev;

#define LAT_HOST_DEV_INLINE static inline

namespace {

// Block -> tile map.  The dispatcher hands block b to XCD b % 8 (each XCD
// has its own L2).  order 0: XCD k owns the z-slab [k*zslab, (k+1)*zslab) for
// every t, so neighbours in x, y and t stay in its L2 and z crosses only at
// the slab faces (the host falls back to order 1 when 8 does not divide Nz
// or work-groups do not tile whole z-planes); 1: identity; 2: reversed;
// 3: one contiguous range of tiles per XCD; 4 (4-D tiles only, see
// thread_site): one z-slab of tiles per XCD.
LAT_DEV int64_t tile_index(int order, int nyb = 1, int zslab = 1, int nz = 1, int reverse = 0) {
    const int64_t nb = gridDim.x, b = blockIdx.x;
    if (order == 1) return b;
    if (order == 2) return nb - 1 - b;
    if (order == 0) {
        const int k = (int)(b & 7);
        int64_t j = b >> 3;
        // walking the slab backwards on every other pass starts a pass on the
        // links the previous pass touched last, still in this XCD's L2
        if (reverse) j = (nb >> 3) - 1 - j;
        const int yb = (int)(j % nyb);
        j /= nyb;
        const int zl = (int)(j % zslab);
        const int64_t t = j / zslab;
        return yb + (int64_t)nyb * ((k * zslab + zl) + (int64_t)nz * t);
    }
    const int64_t x = b & 7, k = b >> 3;
    const int64_t per = nb >> 3, rem = nb & 7;
    return x * per + (x < rem ? x : rem) + k;
}

// Half-lattice index of this thread's site, or -1 if it lies outside the
// lattice.  Lexicographic runs of blockDim sites, or a compact 4-D tile
// (x/2, y, z, t) per work-group so that neighbour links are shared inside
// the work-group and its XCD.
LAT_DEV int64_t thread_site(const PassArgs& a) {
    int bx, by, bz, bt;
    if (a.tshape[0] && a.tile_order == 4) {
        // XCD-blocked 4-D tiles: the tile grid is enumerated x, y, t, then z
        // (slowest), and XCD k (block b runs on XCD b mod 8) takes the k-th
        // contiguous eighth of that list, i.e. a z-slab of tiles, walked in
        // the same order (backwards on every other pass)
        const int64_t nb = gridDim.x, b = blockIdx.x;
        const int64_t k = b & 7, per = nb >> 3, rem = nb & 7;
        int64_t j = b >> 3;
        const int64_t mine = per + (k < rem ? 1 : 0);
        if (a.reverse) j = mine - 1 - j;
        int64_t r = k * per + (k < rem ? k : rem) + j;
        bx = (int)(r % a.tcount[0]);
        r /= a.tcount[0];
        by = (int)(r % a.tcount[1]);
        r /= a.tcount[1];
        bt = (int)(r % a.tcount[3]);
        bz = (int)(r / a.tcount[3]);
    } else {
        const int64_t tile = tile_index(a.tile_order, a.nyb, a.zslab, a.g.nz, a.reverse);
        if (a.tshape[0] == 0) {
            const int64_t s = tile * (int64_t)blockDim.x + threadIdx.x;
            return s < a.g.vh ? s : -1;
        }
        int64_t r = tile;
        bx = (int)(r % a.tcount[0]);
        r /= a.tcount[0];
        by = (int)(r % a.tcount[1]);
        r /= a.tcount[1];
        bz = (int)(r % a.tcount[2]);
        bt = (int)(r / a.tcount[2]);
    }
    int i = threadIdx.x;
    const int ix = i % a.tshape[0];
    i /= a.tshape[0];
    const int iy = i % a.tshape[1];
    i /= a.tshape[1];
    const int iz = i % a.tshape[2];
    const int it = i / a.tshape[2];
    const int xh = bx * a.tshape[0] + ix, y = by * a.tshape[1] + iy;
    const int z = bz * a.tshape[2] + iz, t = bt * a.tshape[3] + it;
    if (xh >= a.g.nxh || y >= a.g.ny || z >= a.g.nz || t >= a.g.nt) return -1;
    return xh + (int64_t)a.g.nxh * (y + (int64_t)a.g.ny * (z + (int64_t)a.g.nz * t));
}

constexpr int SUB_A[3] = {0, 1, 0};
constexpr int SUB_B[3] = {1, 2, 2};

// ---------------------------------------------------------------------------
// SU(3) pass
// ---------------------------------------------------------------------------
// Update of the link U_mu(x) at half-lattice index s of the pass parity.
// MU >= 0 fixes the direction at compile time (the staple then is one
// straight-line block the scheduler can interleave); MU = -1 reads it from
// the arguments.
// ---------------------------------------------------------------------------
// LDS staging of the opposite-parity U_mu links of a 4-D tile
// ---------------------------------------------------------------------------
// A pass reads each link U_mu(y) of the other parity six times (from the
// sites y -+ nu, nu != mu), and those readers are spread over the whole
// staple loop of many work-groups, longer than the per-XCD L2 keeps the
// lines.  With staging, a work-group covers a 4-D tile of the pass parity
// whose extents divide the lattice; it first copies into LDS every U_mu link
// of the other parity that its sites read -- the tile's own box (in x
// widened by one half-site on each side unless mu = x) and one face on each
// side in every other direction nu != mu, x, with periodic wrap-around --
// and then takes those six neighbours from LDS.  Element k of slot j sits at
// lds + (k * nslots + j) * VB, so a wave's reads of consecutive slots are
// contiguous.
struct lq_tile {
    int x0, y0, z0, t0;  // origin (x/2, y, z, t)
    int tx, ty, tz, tt;  // extents
    int ex;              // 1 unless mu = x: the box reaches one half-site further on both x sides
    int nI;              // slots of the box
    int fo[4];           // first slot of the two faces of direction nu (nu = y, z, t; nu != mu)
    int fs[4];           // slots of one face
    int nslots;
};

LAT_DEV lq_tile lq_make(int mu, int bx, int by, int bz, int bt, const int (&sh)[4]) {
    lq_tile T;
    T.tx = sh[0];
    T.ty = sh[1];
    T.tz = sh[2];
    T.tt = sh[3];
    T.x0 = bx * T.tx;
    T.y0 = by * T.ty;
    T.z0 = bz * T.tz;
    T.t0 = bt * T.tt;
    T.ex = mu == 0 ? 0 : 1;
    T.nI = (T.tx + 2 * T.ex) * T.ty * T.tz * T.tt;
    const int vol = T.tx * T.ty * T.tz * T.tt;
    int off = T.nI;
    T.fo[0] = T.fs[0] = 0;
#pragma unroll
    for (int nu = 1; nu < 4; ++nu) {
        const int ext = nu == 1 ? T.ty : nu == 2 ? T.tz : T.tt;
        T.fs[nu] = vol / ext;
        T.fo[nu] = off;
        if (nu != mu) off += 2 * T.fs[nu];
    }
    T.nslots = off;
    return T;
}

LAT_DEV int lq_box(const lq_tile& T, int lxx, int ly, int lz, int lt) {
    return (lxx + T.ex) + (T.tx + 2 * T.ex) * (ly + T.ty * (lz + T.tz * lt));
}

// Slot of U_mu(x + d nu) for the tile-local site (lx, ly, lz, lt) of the pass
// parity; r = the x offset of that site within its pair of x (its row parity).
LAT_DEV int lq_slot(const lq_tile& T, int nu, int d, int lx, int ly, int lz, int lt, int r) {
    switch (nu) {
        case 0: return lq_box(T, lx + (d > 0 ? r : r - 1), ly, lz, lt);
        case 1: {
            const int l = ly + d;
            if (l >= 0 && l < T.ty) return lq_box(T, lx, l, lz, lt);
            return T.fo[1] + (l < 0 ? 0 : T.fs[1]) + lx + T.tx * (lz + T.tz * lt);
        }
        case 2: {
            const int l = lz + d;
            if (l >= 0 && l < T.tz) return lq_box(T, lx, ly, l, lt);
            return T.fo[2] + (l < 0 ? 0 : T.fs[2]) + lx + T.tx * (ly + T.ty * lt);
        }
        default: {
            const int l = lt + d;
            if (l >= 0 && l < T.tt) return lq_box(T, lx, ly, lz, l);
            return T.fo[3] + (l < 0 ? 0 : T.fs[3]) + lx + T.tx * (ly + T.ty * lz);
        }
    }
}

LAT_DEV int wrap(int c, int n) { return c < 0 ? c + n : (c >= n ? c - n : c); }

// Half-lattice index of the link that LDS slot j of the tile holds.
LAT_DEV uint32_t lq_source(const PassArgs& a, const lq_tile& T, int mu, int j) {
    int xh, y, z, t;
    if (j < T.nI) {
        const int w = T.tx + 2 * T.ex;
        int r = j / w;
        xh = T.x0 + (j - r * w) - T.ex;
        y = T.y0 + r % T.ty;
        r /= T.ty;
        z = T.z0 + r % T.tz;
        t = T.t0 + r / T.tz;
    } else {
        int nu = 1;
        while (nu < 3 && (nu == mu || j >= T.fo[nu] + 2 * T.fs[nu])) ++nu;
        const int k = j - T.fo[nu];
        const int side = k >= T.fs[nu];
        const int i = side ? k - T.fs[nu] : k;
        const int lx = i % T.tx;
        const int rest = i / T.tx;
        xh = T.x0 + lx;
        if (nu == 1) {
            y = side ? T.y0 + T.ty : T.y0 - 1;
            z = T.z0 + rest % T.tz;
            t = T.t0 + rest / T.tz;
        } else if (nu == 2) {
            y = T.y0 + rest % T.ty;
            z = side ? T.z0 + T.tz : T.z0 - 1;
            t = T.t0 + rest / T.ty;
        } else {
            y = T.y0 + rest % T.ty;
            z = T.z0 + rest / T.ty;
            t = side ? T.t0 + T.tt : T.t0 - 1;
        }
    }
    xh = wrap(xh, a.g.nxh);
    y = wrap(y, a.g.ny);
    z = wrap(z, a.g.nz);
    t = wrap(t, a.g.nt);
    return (uint32_t)xh + (uint32_t)a.g.nxh * ((uint32_t)y + (uint32_t)a.g.ny * ((uint32_t)z + (uint32_t)a.g.nz * t));
}

// Copies the tile's U_mu links of parity q into LDS (all threads of the
// work-group; the caller synchronises).  A thread's slots are taken
// LQ_FILL at a time and all their loads are issued before the first LDS
// write; slot indices past the end are clamped to the last slot for the
// loads (every load stays inside the lattice) and their writes are
// skipped.  Grouping four slots made the staged overrelaxation pass of the
// FP64 12-real form 23% and of the FP32 18-real form 8% faster on MI355X
// (32^3x8, same run), and those of the FP64 18-real and FP32 12-real forms
// 3% slower: they keep one slot at a time.
template <class ST>
LAT_DEV void lq_fill(const PassArgs& a, const lq_tile& T, int mu, int q, char* lds) {
    using V = typename ST::vec;
    constexpr int LQ_FILL = (std::is_same<ST, st_f64c12>::value || std::is_same<ST, st_f32>::value) ? 4 : 1;
    const char* src = dir_base<ST>(a.links, a.g.vh_pad, q, mu);
    const int64_t pb = a.g.vh_pad * ST::VB;
    for (int j0 = threadIdx.x; j0 < T.nslots; j0 += LQ_FILL * (int)blockDim.x) {
        uint32_t gs[LQ_FILL];
#pragma unroll
        for (int u = 0; u < LQ_FILL; ++u) {
            const int j = j0 + u * (int)blockDim.x;
            gs[u] = lq_source(a, T, mu, j < T.nslots ? j : T.nslots - 1);
        }
        V v[LQ_FILL][ST::NP];
#pragma unroll
        for (int u = 0; u < LQ_FILL; ++u)
#pragma unroll
            for (int k = 0; k < ST::NP; ++k) v[u][k] = ld_plane<V>(src, pb, k, gs[u] * ST::VB);
#pragma unroll
        for (int u = 0; u < LQ_FILL; ++u) {
            const int j = j0 + u * (int)blockDim.x;
            if (j < T.nslots) {
#pragma unroll
                for (int k = 0; k < ST::NP; ++k)
                    *reinterpret_cast<V*>(lds + ((int64_t)k * T.nslots + j) * ST::VB) = v[u][k];
            }
        }
    }
}

// Where this thread's site finds its staged neighbours in an LDS-staged
// pass: the slots of U_mu(x + nu) and U_mu(x - nu) for every nu.
struct lq_site {
    const char* lds = nullptr;
    int nslots = 0;
    int fwd[4] = {0, 0, 0, 0}, bwd[4] = {0, 0, 0, 0};
};

template <class ST, int KIND, bool REUNIT, int RNG, int MU = -1, bool LQ = false>
LAT_DEV void su3_site(const PassArgs& a, int64_t s, const lq_site& lq = lq_site()) {
    using T = typename ST::real;
    using M = m3<T>;
    __shared__ uint32_t rl_lds[RNG == LAT_RNG_RANLUX_I ? 24 * 256 : 1];  // current RANLUX block
    const int p = a.parity, q = 1 - p, mu = MU >= 0 ? MU : a.mu;
    const int64_t vp = a.g.vh_pad;
    const char* L = a.links;
    const site32 cs = site_of(a.g, (uint32_t)s, p);
    const coord4 c = coords(cs);
    if (a.frozen && mu < 3 && c.t == 0) return;  // held at the background field
    const site32 cpm = site_step(a.g, cs, mu, +1);
    const int64_t s_pm = cpm.s;

    int64_t canon = 0;
    draws<RNG> d;
    if constexpr (KIND == 0) {
        canon = canon_index(a.g, c);
        if constexpr (RNG == LAT_RNG_PHILOX_I) {
            d.site = (uint32_t)canon;
            d.lat = a.lat_id;
            d.word2 = (uint32_t)(4 * (*a.hb_count + (uint64_t)a.hb_offset) + mu);
            d.k0 = a.key0;
            d.k1 = a.key1;
            d.nhit = a.nhit;
        } else if constexpr (RNG == LAT_RNG_MRG_I) {
#pragma unroll
            for (int w = 0; w < 6; ++w) d.st.s[w] = a.mrg[((int64_t)p * 6 + w) * vp + s];
        } else if constexpr (RNG == LAT_RNG_RANLUX_I) {
            // every link update begins a new block of the site's stream
            uint32_t b[24];
#pragma unroll
            for (int j = 0; j < 24; ++j) b[j] = a.mrg[((int64_t)p * 25 + j) * vp + s];
            const uint32_t f = a.mrg[((int64_t)p * 25 + 24) * vp + s];
            uint32_t cy = f & 1u;
            ranlux_next_block(b, cy, (f & 2u) == 0);
            d.lds = rl_lds + threadIdx.x;
            d.stride = (int)blockDim.x;
#pragma unroll
            for (int j = 0; j < 24; ++j) d.lds[j * d.stride] = b[j];
            d.c = cy;
            d.idx = 0;
        } else {
            d.c = a.rng_const;
        }
    }
    // counter-addressed and constant draws do not depend on earlier tries
    constexpr bool PREPARE = (KIND == 0 && (RNG == LAT_RNG_PHILOX_I || RNG == LAT_RNG_CONST_I));
    kp_first first[3];

    // staple A = sum_{nu != mu} [U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
    //                           + U_nu(x+mu-nu)^+ U_mu(x-nu)^+ U_nu(x-nu)]
    // The six links of one direction nu are requested together, so that the
    // neighbouring threads that reuse them find the lines still in L2.
    M A = zero3<T>();
#pragma unroll
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        const int64_t s_pn = site_step(a.g, cs, nu, +1).s;
        const int64_t s_mn = site_step(a.g, cs, nu, -1).s;
        const int64_t s_pmmn = site_step(a.g, cpm, nu, -1).s;
        // Two-row products: the first factor of a partial product is used
        // without its third row (for the 12-real forms its third row is not
        // rebuilt, for the 18-real ones not loaded); two rows of the product
        // are formed and the third follows from them (the product is in
        // SU(3)).  Same-run timing on MI355X chose where: 12-real forms in
        // both terms of the heat baths and the FP64 overrelaxation, in the
        // forward term only of the FP32 overrelaxation (2%; both terms 5%
        // slower than neither); 18-real forms in both terms (32^3x8: FP32
        // OR 19.1 -> 17.8 us, FP64 OR 37.7 -> 35.5 us, heat baths 3% faster;
        // 64^3x16 FP64: OR 669 -> 646 us, heat bath 773 -> 718 us).  With
        // them the per-direction overrelaxation kernels lost to those taking
        // the direction at run time for every form but FP32 12-real (FP64
        // 18-real OR 50.7 against 35.5 us; see launch_su3).  Every pass of a
        // form, plain or staged, does the same arithmetic and gives the same
        // links.
        constexpr bool TRF = true;
        constexpr bool TRB = !ST::TWO_ROWS || KIND == 0 || std::is_same<T, double>::value;
        // In the FP64 12-real heat bath the forward term is loaded and
        // accumulated before the backward term's links are requested, with
        // scheduling barriers that keep the compiler from hoisting them:
        // three links live instead of six (195 registers instead of 292, two
        // waves per SIMD instead of one; 32^3x8 heat-bath pass 38.2 ->
        // 34.9 us on MI355X, same run).  Every other pass requests all six
        // links first (most loads in flight); for them the split was slower.
        constexpr bool SPLIT = KIND == 0 && std::is_same<ST, st_f64c12>::value;
        if constexpr (SPLIT) {
            const M f0 = load_link_rows01<ST>(L, vp, q, nu, s_pm);
            const M f1 = [&] {  // U_mu(x + nu): staged in LDS or from memory
                if constexpr (LQ) return ST::load(lq.lds, lq.nslots, lq.fwd[nu]);
                else return load_link<ST>(L, vp, q, mu, s_pn);
            }();
            const M f2 = load_link<ST>(L, vp, p, nu, s);
            if constexpr (PREPARE) {
                if (nu == (mu == 0 ? 1 : 0)) {
#pragma unroll
                    for (int g = 0; g < 3; ++g) first[g] = kp_prepare(d, g);
                }
            }
            M fq;
            mul_na_rows01(fq, f0, f1);
            third_row(fq);
            mac_na(A, fq, f2);
            __builtin_amdgcn_sched_barrier(0);
            const M b0 = [&] {  // U_mu(x - nu)
                if constexpr (LQ) return ST::load_rows01(lq.lds, lq.nslots, lq.bwd[nu]);
                else return load_link_rows01<ST>(L, vp, q, mu, s_mn);
            }();
            const M b1 = load_link<ST>(L, vp, p, nu, s_pmmn);
            const M b2 = load_link<ST>(L, vp, q, nu, s_mn);
            M bq;
            mul_nn_rows01(bq, b0, b1);
            third_row(bq);
            mac_an(A, bq, b2);
            __builtin_amdgcn_sched_barrier(0);
        } else {
            const M f0 = [&] {
                if constexpr (TRF) return load_link_rows01<ST>(L, vp, q, nu, s_pm);
                else return load_link<ST>(L, vp, q, nu, s_pm);
            }();
            const M f1 = [&] {  // U_mu(x + nu): staged in LDS or from memory
                if constexpr (LQ) return ST::load(lq.lds, lq.nslots, lq.fwd[nu]);
                else return load_link<ST>(L, vp, q, mu, s_pn);
            }();
            const M f2 = load_link<ST>(L, vp, p, nu, s);
            const M b0 = [&] {  // U_mu(x - nu)
                if constexpr (LQ && TRB) return ST::load_rows01(lq.lds, lq.nslots, lq.bwd[nu]);
                else if constexpr (LQ) return ST::load(lq.lds, lq.nslots, lq.bwd[nu]);
                else if constexpr (TRB) return load_link_rows01<ST>(L, vp, q, mu, s_mn);
                else return load_link<ST>(L, vp, q, mu, s_mn);
            }();
            const M b1 = load_link<ST>(L, vp, p, nu, s_pmmn);
            const M b2 = load_link<ST>(L, vp, q, nu, s_mn);
            if constexpr (PREPARE) {
                // while the first direction's links are in flight, turn the
                // random numbers of each subgroup's first try into its candidate
                if (nu == (mu == 0 ? 1 : 0)) {
#pragma unroll
                    for (int g = 0; g < 3; ++g) first[g] = kp_prepare(d, g);
                }
            }
            if constexpr (TRF) {
                M fq;
                mul_na_rows01(fq, f0, f1);
                third_row(fq);
                mac_na(A, fq, f2);
            } else {
                mac_na(A, mul_na(f0, f1), f2);
            }
            if constexpr (TRB) {
                M bq;
                mul_nn_rows01(bq, b0, b1);
                third_row(bq);
                mac_an(A, bq, b2);
            } else {
                mac_an(A, mul_nn(b0, b1), b2);
            }
        }
    }
    M U = load_link<ST>(L, vp, p, mu, s);
    M W = mul_nn(U, A);  // link times staple: the local action is Re Tr(W)

#pragma unroll
    for (int g = 0; g < 3; ++g) {
        const int ia = SUB_A[g], ib = SUB_B[g];
        const qt<T> qb = block_quat(W, ia, ib);
        qt<T> rt;
        if constexpr (KIND == 1 && std::is_same<T, float>::value) {
            // FP32 forms: r = (v^+)^2 with v = q/|q| is q^+ q^+ / |q|^2, so
            // no square root is needed.  Products of two FP32 numbers are
            // exact in FP64; the numerators and |q|^2 are formed in FP64,
            // 1/|q|^2 is the hardware reciprocal refined by one Newton step
            // (relative error ~1e-16), and r is rounded to FP32 once, as
            // when it is computed from v in FP64.
            const double q0 = qb.q0, q1 = qb.q1, q2 = qb.q2, q3 = qb.q3;
            const double n2 = q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3;
            if (!(n2 > 0.0)) continue;
            const double i0 = __builtin_amdgcn_rcp(n2);
            const double inv = fma(i0, fma(-n2, i0, 1.0), i0);
            const double m2 = -2.0 * q0 * inv;
            rt = {(float)((q0 * q0 - (q1 * q1 + q2 * q2 + q3 * q3)) * inv), (float)(m2 * q1), (float)(m2 * q2),
                  (float)(m2 * q3)};
        } else {
            const qt<double> qd = {(double)qb.q0, (double)qb.q1, (double)qb.q2, (double)qb.q3};
            const double k = sqrt(qnorm2(qd));
            qt<double> r;
            if constexpr (KIND == 0) {
                const double alpha = 2.0 * a.beta * k / 3.0;
                int8_t* log = a.accept_log ? a.accept_log + ((((int64_t)a.hb_offset * 4 + mu) * (2 * a.g.vh) + canon) * 3 + g) : nullptr;
                if (!(alpha >= 1e-12)) {
                    if (log) *log = -1;
                    continue;
                }
                qt<double> x;
                int t;
                if constexpr (PREPARE) t = kp_prepared(alpha, a.nhit, d, g, first[g], x);
                else t = kp(alpha, a.nhit, d, g, x);
                if (log) *log = (int8_t)t;
                if (t < 0) continue;
                const double ik = 1.0 / k;
                r = qmul_na(x, qt<double>{qd.q0 * ik, qd.q1 * ik, qd.q2 * ik, qd.q3 * ik});
            } else {
                if (!(k > 0.0)) continue;
                const double ik = 1.0 / k;
                const qt<double> vd = {qd.q0 * ik, -qd.q1 * ik, -qd.q2 * ik, -qd.q3 * ik};
                r = qmul(vd, vd);
            }
            rt = {(T)r.q0, (T)r.q1, (T)r.q2, (T)r.q3};
        }
        left_mul_block(U, ia, ib, rt);
        if (g < 2) left_mul_block(W, ia, ib, rt);
    }

    if constexpr (REUNIT) {
        m3<double> ud = cast3<double>(U);
        reunit3(ud);
        U = cast3<T>(ud);
    }
    ST::store(const_cast<char*>(dir_base<ST>(L, vp, p, mu)), vp, s, U);
    if constexpr (KIND == 0 && RNG == LAT_RNG_MRG_I) {
#pragma unroll
        for (int w = 0; w < 6; ++w) a.mrg[((int64_t)p * 6 + w) * vp + s] = d.st.s[w];
    }
    if constexpr (KIND == 0 && RNG == LAT_RNG_RANLUX_I) {
#pragma unroll
        for (int j = 0; j < 24; ++j) a.mrg[((int64_t)p * 25 + j) * vp + s] = d.lds[j * d.stride];
        a.mrg[((int64_t)p * 25 + 24) * vp + s] = d.c;  // a block has been delivered
    }
}

// The last overrelaxation pass of a compound sweep also advances the
// heat-bath counter (no pass that reads it runs before this kernel ends).
LAT_DEV void pass_bump(const PassArgs& a) {
    if (a.bump_by != 0 && blockIdx.x == 0 && threadIdx.x == 0) *a.bump_counter += (uint64_t)a.bump_by;
}

template <class ST, int KIND, bool REUNIT, int RNG, int MU>
__global__ void __launch_bounds__(256) su3_pass(PassArgs a) {
    const int64_t s = thread_site(a);
    if (s >= 0) su3_site<ST, KIND, REUNIT, RNG, MU>(a, s);
    if constexpr (KIND == 1) pass_bump(a);
}

// The same pass with the tile's opposite-parity U_mu links staged in LDS
// (4-D tiles that divide the lattice; the host checks both).
template <class ST, int KIND, bool REUNIT, int RNG, int MU>
__global__ void __launch_bounds__(256) su3_pass_lq(PassArgs a) {
    extern __shared__ __align__(16) char lq_lds[];
    int bx, by, bz, bt;
    if (a.tile_order == 4) {
        const int64_t nb = gridDim.x, b = blockIdx.x;
        const int64_t k = b & 7, per = nb >> 3, rem = nb & 7;
        int64_t j = b >> 3;
        const int64_t mine = per + (k < rem ? 1 : 0);
        if (a.reverse) j = mine - 1 - j;
        int64_t r = k * per + (k < rem ? k : rem) + j;
        bx = (int)(r % a.tcount[0]);
        r /= a.tcount[0];
        by = (int)(r % a.tcount[1]);
        r /= a.tcount[1];
        bt = (int)(r % a.tcount[3]);
        bz = (int)(r / a.tcount[3]);
    } else {
        int64_t r = blockIdx.x;
        bx = (int)(r % a.tcount[0]);
        r /= a.tcount[0];
        by = (int)(r % a.tcount[1]);
        r /= a.tcount[1];
        bz = (int)(r % a.tcount[2]);
        bt = (int)(r / a.tcount[2]);
    }
    const int mu = MU >= 0 ? MU : a.mu;
    const lq_tile T = lq_make(mu, bx, by, bz, bt, a.tshape);
    lq_fill<ST>(a, T, mu, 1 - a.parity, lq_lds);
    __syncthreads();
    int i = threadIdx.x;
    const int lx = i % T.tx;
    i /= T.tx;
    const int ly = i % T.ty;
    i /= T.ty;
    const int lz = i % T.tz;
    const int lt = i / T.tz;
    const int y = T.y0 + ly, z = T.z0 + lz, t = T.t0 + lt;
    const int r = (a.parity + y + z + t) & 1;  // x = 2 (x0 + lx) + r
    lq_site ls;
    ls.lds = lq_lds;
    ls.nslots = T.nslots;
#pragma unroll
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        ls.fwd[nu] = lq_slot(T, nu, +1, lx, ly, lz, lt, r);
        ls.bwd[nu] = lq_slot(T, nu, -1, lx, ly, lz, lt, r);
    }
    const int64_t s = (T.x0 + lx) + (int64_t)a.g.nxh * (y + (int64_t)a.g.ny * (z + (int64_t)a.g.nz * t));
    su3_site<ST, KIND, REUNIT, RNG, MU, true>(a, s, ls);
    if constexpr (KIND == 1) pass_bump(a);
}

// ---------------------------------------------------------------------------
// SU(2) pass (quaternions)
// ---------------------------------------------------------------------------
// Update of the link U_mu(x) at half-lattice index s of the pass parity.
template <class ST, int KIND, bool REUNIT, int RNG>
LAT_DEV void su2_site(const PassArgs& a, int64_t s) {
    using T = typename ST::real;
    using Q = qt<T>;
    __shared__ uint32_t rl_lds[RNG == LAT_RNG_RANLUX_I ? 24 * 256 : 1];  // current RANLUX block
    const int p = a.parity, q = 1 - p, mu = a.mu;
    const int64_t vp = a.g.vh_pad;
    const char* L = a.links;
    const site32 cs = site_of(a.g, (uint32_t)s, p);
    const coord4 c = coords(cs);
    if (a.frozen && mu < 3 && c.t == 0) return;  // held at the background field
    const site32 cpm = site_step(a.g, cs, mu, +1);
    const int64_t s_pm = cpm.s;

    Q A = {T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        const int64_t s_pn = site_step(a.g, cs, nu, +1).s;
        const int64_t s_mn = site_step(a.g, cs, nu, -1).s;
        const int64_t s_pmmn = site_step(a.g, cpm, nu, -1).s;
        Q f = qmul_na(qmul_na(load_link<ST>(L, vp, q, nu, s_pm), load_link<ST>(L, vp, q, mu, s_pn)),
                      load_link<ST>(L, vp, p, nu, s));
        A = qadd(A, f);
        Q b = qmul(qdag(qmul(load_link<ST>(L, vp, q, mu, s_mn), load_link<ST>(L, vp, p, nu, s_pmmn))),
                   load_link<ST>(L, vp, q, nu, s_mn));
        A = qadd(A, b);
    }
    Q U = load_link<ST>(L, vp, p, mu, s);
    const Q W = qmul(U, A);
    const qt<double> qd = {(double)W.q0, (double)W.q1, (double)W.q2, (double)W.q3};
    const double k = sqrt(qnorm2(qd));
    bool apply = false;
    qt<double> r;
    if constexpr (KIND == 0) {
        const int64_t canon = canon_index(a.g, c);
        draws<RNG> d;
        if constexpr (RNG == LAT_RNG_PHILOX_I) {
            d.site = (uint32_t)canon;
            d.lat = a.lat_id;
            d.word2 = (uint32_t)(4 * (*a.hb_count + (uint64_t)a.hb_offset) + mu);
            d.k0 = a.key0;
            d.k1 = a.key1;
            d.nhit = a.nhit;
        } else if constexpr (RNG == LAT_RNG_MRG_I) {
#pragma unroll
            for (int w = 0; w < 6; ++w) d.st.s[w] = a.mrg[((int64_t)p * 6 + w) * vp + s];
        } else if constexpr (RNG == LAT_RNG_RANLUX_I) {
            uint32_t b[24];
#pragma unroll
            for (int j = 0; j < 24; ++j) b[j] = a.mrg[((int64_t)p * 25 + j) * vp + s];
            const uint32_t f = a.mrg[((int64_t)p * 25 + 24) * vp + s];
            uint32_t cy = f & 1u;
            ranlux_next_block(b, cy, (f & 2u) == 0);
            d.lds = rl_lds + threadIdx.x;
            d.stride = (int)blockDim.x;
#pragma unroll
            for (int j = 0; j < 24; ++j) d.lds[j * d.stride] = b[j];
            d.c = cy;
            d.idx = 0;
        } else {
            d.c = a.rng_const;
        }
        const double alpha = 2.0 * a.beta * k / 2.0;
        int8_t* log = a.accept_log ? a.accept_log + ((((int64_t)a.hb_offset * 4 + mu) * (2 * a.g.vh) + canon) * 3) : nullptr;
        if (alpha >= 1e-12) {
            qt<double> x;
            const int t = kp(alpha, a.nhit, d, 0, x);
            if (log) *log = (int8_t)t;
            if (t >= 0) {
                const double ik = 1.0 / k;
                r = qmul_na(x, qt<double>{qd.q0 * ik, qd.q1 * ik, qd.q2 * ik, qd.q3 * ik});
                apply = true;
            }
        } else if (log) {
            *log = -1;
        }
        if constexpr (RNG == LAT_RNG_MRG_I) {
#pragma unroll
            for (int w = 0; w < 6; ++w) a.mrg[((int64_t)p * 6 + w) * vp + s] = d.st.s[w];
        }
        if constexpr (RNG == LAT_RNG_RANLUX_I) {
#pragma unroll
            for (int j = 0; j < 24; ++j) a.mrg[((int64_t)p * 25 + j) * vp + s] = d.lds[j * d.stride];
            a.mrg[((int64_t)p * 25 + 24) * vp + s] = d.c;
        }
    } else if constexpr (std::is_same<T, float>::value) {
        // FP32 storage: r = q^+ q^+ / |q|^2 from the exact FP64 products of
        // the FP32 components, rounded to FP32 once (as for SU(3))
        const double n2 = qd.q0 * qd.q0 + qd.q1 * qd.q1 + qd.q2 * qd.q2 + qd.q3 * qd.q3;
        if (n2 > 0.0) {
            const double i0 = __builtin_amdgcn_rcp(n2);
            const double inv = fma(i0, fma(-n2, i0, 1.0), i0);
            const double m2 = -2.0 * qd.q0 * inv;
            r = {(qd.q0 * qd.q0 - (qd.q1 * qd.q1 + qd.q2 * qd.q2 + qd.q3 * qd.q3)) * inv, m2 * qd.q1, m2 * qd.q2,
                 m2 * qd.q3};
            apply = true;
        }
    } else {
        if (k > 0.0) {
            const double ik = 1.0 / k;
            const qt<double> vd = {qd.q0 * ik, -qd.q1 * ik, -qd.q2 * ik, -qd.q3 * ik};
            r = qmul(vd, vd);
            apply = true;
        }
    }
    if (apply) U = qmul(Q{(T)r.q0, (T)r.q1, (T)r.q2, (T)r.q3}, U);
    if constexpr (REUNIT) {
        qt<double> ud = {(double)U.q0, (double)U.q1, (double)U.q2, (double)U.q3};
        const double in = 1.0 / sqrt(qnorm2(ud));
        U = {(T)(ud.q0 * in), (T)(ud.q1 * in), (T)(ud.q2 * in), (T)(ud.q3 * in)};
    }
    ST::store(const_cast<char*>(dir_base<ST>(L, vp, p, mu)), vp, s, U);
}

template <class ST, int KIND, bool REUNIT, int RNG>
__global__ void __launch_bounds__(256) su2_pass(PassArgs a) {
    const int64_t s = thread_site(a);
    if (s >= 0) su2_site<ST, KIND, REUNIT, RNG>(a, s);
    if constexpr (KIND == 1) pass_bump(a);
}

// ---------------------------------------------------------------------------
// initialisation: cold (unit) or Haar-random links, times the background
// ---------------------------------------------------------------------------
// RANLUX state of one site during initialisation: every link's draws begin
// a new block (the values are taken in order, so registers suffice).
struct ranlux_init {
    uint32_t b[24];
    uint32_t c;
    bool first;
    LAT_DEV void load(const uint32_t* st, int64_t vp, int p, int64_t s) {
#pragma unroll
        for (int j = 0; j < 24; ++j) b[j] = st[((int64_t)p * 25 + j) * vp + s];
        const uint32_t f = st[((int64_t)p * 25 + 24) * vp + s];
        c = f & 1u;
        first = (f & 2u) != 0;
    }
    LAT_DEV void draw(double* u, int n) {
        ranlux_next_block(b, c, !first);
        first = false;
        for (int k = 0; k < n; ++k) u[k] = u24(b[k] << 8);
    }
    LAT_DEV void store(uint32_t* st, int64_t vp, int p, int64_t s) const {
#pragma unroll
        for (int j = 0; j < 24; ++j) st[((int64_t)p * 25 + j) * vp + s] = b[j];
        st[((int64_t)p * 25 + 24) * vp + s] = c | (first ? 2u : 0u);
    }
};

LAT_DEV void box_muller(double u1, double u2, double& g1, double& g2) {
    const double r = sqrt(-2.0 * log(u1));
    double sn, cs;
    sincos(TWO_PI * u2, &sn, &cs);
    g1 = r * cs;
    g2 = r * sn;
}

template <int RNG>
LAT_DEV void init_uniforms(const InitArgs& a, int64_t canon, int mu, int nu, double* u, mrg_state& st) {
    if constexpr (RNG == LAT_RNG_PHILOX_I) {
        for (int j = 0; j < nu / 4; ++j) {
            u4 o = philox10({(uint32_t)canon, a.lat_id, 0xFFFFFFFFu, (uint32_t)(4 * mu + j)}, a.key0, a.key1);
            u[4 * j] = u24(o.x);
            u[4 * j + 1] = u24(o.y);
            u[4 * j + 2] = u24(o.z);
            u[4 * j + 3] = u24(o.w);
        }
    } else if constexpr (RNG == LAT_RNG_MRG_I) {
        for (int k = 0; k < nu; ++k) u[k] = u24(mrg_step(st));
    } else {
        for (int k = 0; k < nu; ++k) u[k] = a.rng_const;
    }
}

template <class ST, int RNG>
__global__ void __launch_bounds__(256) su3_init(InitArgs a) {
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int p = blockIdx.y;
    if (s >= a.g.vh) return;
    const int64_t vp = a.g.vh_pad;
    const coord4 c = decode(a.g, s, p);
    const int64_t canon = canon_index(a.g, c);
    mrg_state st;
    ranlux_init rl;
    if constexpr (RNG == LAT_RNG_MRG_I) {
        for (int w = 0; w < 6; ++w) st.s[w] = a.mrg[((int64_t)p * 6 + w) * vp + s];
    }
    if constexpr (RNG == LAT_RNG_RANLUX_I) rl.load(a.mrg, vp, p, s);
    for (int mu = 0; mu < 4; ++mu) {
        m3<double> U = identity3<double>();
        if (a.start == 1) {
            double u[12];
            if constexpr (RNG == LAT_RNG_RANLUX_I) rl.draw(u, 12);
            else init_uniforms<RNG>(a, canon, mu, 12, u, st);
#pragma unroll
            for (int row = 0; row < 2; ++row)
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) {
                    double re, im;
                    box_muller(u[6 * row + 2 * cc], u[6 * row + 2 * cc + 1], re, im);
                    U.e[row][cc] = {re, im};
                }
            reunit3(U);
        }
        if (a.frozen && mu < 3 && c.t == 0) U = identity3<double>();  // W = B
        const double th = bg_theta(a.g, a.flux, c, mu);
        if (th != 0.0) {
            double sn, cs;
            sincos(th, &sn, &cs);
            const cx<double> e = {cs, sn}, ec = {cs, -sn};
            for (int r = 0; r < 3; ++r) {
                U.e[r][0] = cmul(U.e[r][0], e);
                U.e[r][1] = cmul(U.e[r][1], ec);
            }
        }
        ST::store(const_cast<char*>(dir_base<ST>(a.links, vp, p, mu)), vp, s, cast3<typename ST::real>(U));
    }
    if constexpr (RNG == LAT_RNG_MRG_I) {
        for (int w = 0; w < 6; ++w) a.mrg[((int64_t)p * 6 + w) * vp + s] = st.s[w];
    }
    if constexpr (RNG == LAT_RNG_RANLUX_I) {
        if (a.start == 1) rl.store(a.mrg, vp, p, s);
    }
}

template <class ST, int RNG>
__global__ void __launch_bounds__(256) su2_init(InitArgs a) {
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int p = blockIdx.y;
    if (s >= a.g.vh) return;
    const int64_t vp = a.g.vh_pad;
    const coord4 c = decode(a.g, s, p);
    const int64_t canon = canon_index(a.g, c);
    mrg_state st;
    ranlux_init rl;
    if constexpr (RNG == LAT_RNG_MRG_I) {
        for (int w = 0; w < 6; ++w) st.s[w] = a.mrg[((int64_t)p * 6 + w) * vp + s];
    }
    if constexpr (RNG == LAT_RNG_RANLUX_I) rl.load(a.mrg, vp, p, s);
    for (int mu = 0; mu < 4; ++mu) {
        qt<double> U = {1.0, 0.0, 0.0, 0.0};
        if (a.start == 1) {
            double u[4], g[4];
            if constexpr (RNG == LAT_RNG_RANLUX_I) rl.draw(u, 4);
            else init_uniforms<RNG>(a, canon, mu, 4, u, st);
            box_muller(u[0], u[1], g[0], g[1]);
            box_muller(u[2], u[3], g[2], g[3]);
            const double nn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2] + g[3] * g[3]);
            U = {g[0] / nn, g[1] / nn, g[2] / nn, g[3] / nn};
        }
        if (a.frozen && mu < 3 && c.t == 0) U = {1.0, 0.0, 0.0, 0.0};  // W = B
        const double th = bg_theta(a.g, a.flux, c, mu);
        if (th != 0.0) {
            double sn, cs;
            sincos(th, &sn, &cs);
            U = qmul(U, qt<double>{cs, 0.0, 0.0, sn});
        }
        using T = typename ST::real;
        ST::store(const_cast<char*>(dir_base<ST>(a.links, vp, p, mu)), vp, s, qt<T>{(T)U.q0, (T)U.q1, (T)U.q2, (T)U.q3});
    }
    if constexpr (RNG == LAT_RNG_MRG_I) {
        for (int w = 0; w < 6; ++w) a.mrg[((int64_t)p * 6 + w) * vp + s] = st.s[w];
    }
    if constexpr (RNG == LAT_RNG_RANLUX_I) {
        if (a.start == 1) rl.store(a.mrg, vp, p, s);
    }
}

// ---------------------------------------------------------------------------
// observables: per-block FP64 partials (wave shuffle, then LDS across the
// 4 waves of a block), then one block folds the partials with Neumaier
// compensation in a fixed order.
// ---------------------------------------------------------------------------
template <int NV>
LAT_DEV void block_reduce_store(double (&v)[NV], double* out, int64_t stride, int64_t slot) {
    __shared__ double sh[NV][4];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double x = v[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
        v[k] = x;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) sh[k][wave] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double x = 0.0;
            for (int w = 0; w < nw; ++w) x += sh[k][w];
            out[k * stride + slot] = x;
        }
    }
}

// Work-group -> (tile, parity) of the plaquette sum: both parities of a
// tile run on the same XCD (blocks b and b+8) right after each other, so the
// links one parity reads as neighbours are still in L2 for the other.  The
// grid is padded to whole groups of 16; padding blocks contribute nothing.
LAT_DEV void plaq_block(const MeasArgs& a, int& tile, int& parity) {
    const int b = blockIdx.x;
    if (a.zslab) {
        // XCD k (work-group b runs on XCD b mod 8) takes z-slab k, both
        // parities of a region in turn, as the pass kernels do
        const int k = b & 7;
        int j = b >> 3;
        parity = j & 1;
        j >>= 1;
        const int yb = j % a.nyb;
        j /= a.nyb;
        const int zl = j % a.zslab;
        const int t = j / a.zslab;
        tile = yb + a.nyb * ((k * a.zslab + zl) + a.g.nz * t);
        return;
    }
    tile = ((b >> 4) << 3) | (b & 7);
    parity = (b >> 3) & 1;
    if (tile >= a.nb_plaq) tile = -1;
}

template <class ST>
__global__ void __launch_bounds__(256) su3_plaq(MeasArgs a) {
    using T = typename ST::real;
    using M = m3<T>;
    int tile, p;
    plaq_block(a, tile, p);
    const int q = 1 - p;
    const int64_t s = tile < 0 ? a.g.vh : tile * (int64_t)blockDim.x + threadIdx.x;
    double v[2] = {0.0, 0.0};
    if (s < a.g.vh) {
        const int64_t vp = a.g.vh_pad;
        const site32 c = site_of(a.g, (uint32_t)s, p);
#pragma unroll
        for (int mu = 0; mu < 3; ++mu) {
            const int64_t s_pm = site_step(a.g, c, mu, +1).s;
            const M umu = load_link<ST>(a.links, vp, p, mu, s);
#pragma unroll
            for (int nu = mu + 1; nu < 4; ++nu) {
                const int64_t s_pn = site_step(a.g, c, nu, +1).s;
                // Re Tr[(U_mu(x) U_nu(x+mu)) (U_nu(x) U_mu(x+nu))^+]
                const M left = mul_nn(umu, load_link<ST>(a.links, vp, q, nu, s_pm));
                const M right = mul_nn(load_link<ST>(a.links, vp, p, nu, s), load_link<ST>(a.links, vp, q, mu, s_pn));
                const double tr = (double)re_tr_na(left, right) * (1.0 / 3.0);
                v[nu == 3 ? 1 : 0] += tr;
            }
        }
    }
    if (tile >= 0) block_reduce_store<2>(v, a.partial, 2 * (int64_t)a.nb_plaq, (int64_t)p * a.nb_plaq + tile);
}

template <class ST>
__global__ void __launch_bounds__(256) su2_plaq(MeasArgs a) {
    using T = typename ST::real;
    using Q = qt<T>;
    int tile, p;
    plaq_block(a, tile, p);
    const int q = 1 - p;
    const int64_t s = tile < 0 ? a.g.vh : tile * (int64_t)blockDim.x + threadIdx.x;
    double v[2] = {0.0, 0.0};
    if (s < a.g.vh) {
        const int64_t vp = a.g.vh_pad;
        const site32 c = site_of(a.g, (uint32_t)s, p);
#pragma unroll
        for (int mu = 0; mu < 3; ++mu) {
            const int64_t s_pm = site_step(a.g, c, mu, +1).s;
            const Q umu = load_link<ST>(a.links, vp, p, mu, s);
#pragma unroll
            for (int nu = mu + 1; nu < 4; ++nu) {
                const int64_t s_pn = site_step(a.g, c, nu, +1).s;
                const Q left = qmul(umu, load_link<ST>(a.links, vp, q, nu, s_pm));
                const Q right = qmul(load_link<ST>(a.links, vp, p, nu, s), load_link<ST>(a.links, vp, q, mu, s_pn));
                // (1/2) Re Tr(left right^+) = scalar part of left * right^dagger
                const double tr = (double)(left.q0 * right.q0 + left.q1 * right.q1 + left.q2 * right.q2 + left.q3 * right.q3);
                v[nu == 3 ? 1 : 0] += tr;
            }
        }
    }
    if (tile >= 0) block_reduce_store<2>(v, a.partial, 2 * (int64_t)a.nb_plaq, (int64_t)p * a.nb_plaq + tile);
}

// Polyakov loop: a work-group covers 64 spatial sites; wave c multiplies the
// temporal links of t-chunk c (t in [c Nt/4, (c+1) Nt/4)) of each site, and
// wave 0 multiplies the four partial products in order, so the dependent
// chain of loads and products is a quarter of Nt long.
template <class T>
LAT_DEV void poly_mul(m3<T>& P, const m3<T>& U) { P = mul_nn(P, U); }
template <class T>
LAT_DEV void poly_mul(qt<T>& P, const qt<T>& U) { P = qmul(P, U); }
template <class T>
LAT_DEV void poly_set_one(m3<T>& P) { P = identity3<T>(); }
template <class T>
LAT_DEV void poly_set_one(qt<T>& P) { P = {T(1), T(0), T(0), T(0)}; }
template <class T>
LAT_DEV void poly_trace(const m3<T>& P, double v[2]) {
    v[0] = ((double)P.e[0][0].re + (double)P.e[1][1].re + (double)P.e[2][2].re) * (1.0 / 3.0);
    v[1] = ((double)P.e[0][0].im + (double)P.e[1][1].im + (double)P.e[2][2].im) * (1.0 / 3.0);
}
template <class T>
LAT_DEV void poly_trace(const qt<T>& P, double v[2]) {
    v[0] = (double)P.q0;  // (1/2) Tr of an SU(2) element is real
    v[1] = 0.0;
}

template <class ST>
__global__ void __launch_bounds__(256) lat_poly(MeasArgs a) {
    using Mat = typename ST::mat;
    __shared__ Mat part[3][64];
    const int c = threadIdx.x >> 6, i = threadIdx.x & 63;
    const int64_t xs = blockIdx.x * (int64_t)64 + i;
    const int64_t vs = (int64_t)a.g.nx * a.g.ny * a.g.nz;
    Mat P;
    poly_set_one(P);
    int x = 0, y = 0, z = 0;
    if (xs < vs) {
        x = (int)(xs % a.g.nx);
        y = (int)((xs / a.g.nx) % a.g.ny);
        z = (int)(xs / ((int64_t)a.g.nx * a.g.ny));
        const int t0 = (c * a.g.nt) / 4, t1 = ((c + 1) * a.g.nt) / 4;
        for (int t = t0; t < t1; ++t) {
            const coord4 cc = {x, y, z, t};
            poly_mul(P, load_link<ST>(a.links, a.g.vh_pad, (x + y + z + t) & 1, 3, half_index(a.g, cc)));
        }
    }
    if (c > 0) part[c - 1][i] = P;
    __syncthreads();
    double v[2] = {0.0, 0.0};
    if (c == 0 && xs < vs) {
#pragma unroll
        for (int k = 0; k < 3; ++k) poly_mul(P, part[k][i]);
        poly_trace(P, v);
    }
    block_reduce_store<2>(v, a.partial + 4 * (int64_t)a.nb_plaq, a.nb_poly, blockIdx.x);
}

// Neumaier-compensated fold of the partials in a fixed order.
struct nsum {
    double s, c;
};
LAT_DEV nsum nadd(nsum a, double x) {
    const double t = a.s + x;
    a.c += (fabs(a.s) >= fabs(x)) ? (a.s - t) + x : (x - t) + a.s;
    a.s = t;
    return a;
}
LAT_DEV nsum nmerge(nsum a, nsum b) {
    a = nadd(a, b.s);
    a.c += b.c;
    return a;
}

__global__ void __launch_bounds__(256) meas_final(MeasArgs a, double* out, uint32_t* slot_counter) {
    __shared__ nsum sh[4][256];
    const int tid = threadIdx.x;
    const int64_t n[4] = {2 * (int64_t)a.nb_plaq, 2 * (int64_t)a.nb_plaq, a.nb_poly, a.nb_poly};
    const double* src[4] = {a.partial, a.partial + 2 * (int64_t)a.nb_plaq, a.partial + 4 * (int64_t)a.nb_plaq,
                            a.partial + 4 * (int64_t)a.nb_plaq + a.nb_poly};
    // each thread sums its partials i = tid, tid + 256, ... in that order;
    // eight of them are loaded before the first is added, so the loads are
    // in flight together instead of one at a time
    constexpr int U = 8;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        nsum acc = {0.0, 0.0};
        for (int64_t i0 = tid; i0 < n[k]; i0 += 256 * U) {
            double v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t i = i0 + 256 * u;
                v[u] = i < n[k] ? src[k][i] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (i0 + 256 * u < n[k]) acc = nadd(acc, v[u]);
        }
        sh[k][tid] = acc;
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w)
#pragma unroll
            for (int k = 0; k < 4; ++k) sh[k][tid] = nmerge(sh[k][tid], sh[k][tid + w]);
        __syncthreads();
    }
    if (tid == 0) {
        const double V = 2.0 * (double)a.g.vh;
        const double vs = (double)a.g.nx * a.g.ny * a.g.nz;
        const double ps = (sh[0][0].s + sh[0][0].c) / (3.0 * V);
        const double pt = (sh[1][0].s + sh[1][0].c) / (3.0 * V);
        uint32_t slot = 0;
        if (slot_counter) slot = *slot_counter;
        double* o = out + 5 * (int64_t)slot;
        o[0] = 0.5 * (ps + pt);
        o[1] = ps;
        o[2] = pt;
        o[3] = (sh[2][0].s + sh[2][0].c) / vs;
        o[4] = (sh[3][0].s + sh[3][0].c) / vs;
        if (slot_counter) *slot_counter = slot + 1;
    }
}

// ---------------------------------------------------------------------------
// canonical FP64 <-> device layout
// ---------------------------------------------------------------------------
template <class ST, int NG>
__global__ void __launch_bounds__(256) to_device(LatGeom g, const double* canon, char* links) {
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int p = blockIdx.y;
    if (s >= g.vh) return;
    const int64_t i = canon_index(g, decode(g, s, p));
    using T = typename ST::real;
    for (int mu = 0; mu < 4; ++mu) {
        char* base = const_cast<char*>(dir_base<ST>(links, g.vh_pad, p, mu));
        if constexpr (NG == 3) {
            const double* src = canon + (i * 4 + mu) * 18;
            m3<T> m;
            for (int k = 0; k < 9; ++k) m.e[k / 3][k % 3] = {(T)src[2 * k], (T)src[2 * k + 1]};
            ST::store(base, g.vh_pad, s, m);
        } else {
            const double* src = canon + (i * 4 + mu) * 4;
            ST::store(base, g.vh_pad, s, qt<T>{(T)src[0], (T)src[1], (T)src[2], (T)src[3]});
        }
    }
}

template <class ST, int NG>
__global__ void __launch_bounds__(256) to_canonical(LatGeom g, const char* links, double* canon) {
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int p = blockIdx.y;
    if (s >= g.vh) return;
    const int64_t i = canon_index(g, decode(g, s, p));
    for (int mu = 0; mu < 4; ++mu) {
        const typename ST::mat m = load_link<ST>(links, g.vh_pad, p, mu, s);
        if constexpr (NG == 3) {
            double* dst = canon + (i * 4 + mu) * 18;
            for (int k = 0; k < 9; ++k) {
                dst[2 * k] = (double)m.e[k / 3][k % 3].re;
                dst[2 * k + 1] = (double)m.e[k / 3][k % 3].im;
            }
        } else {
            double* dst = canon + (i * 4 + mu) * 4;
            dst[0] = (double)m.q0;
            dst[1] = (double)m.q1;
            dst[2] = (double)m.q2;
            dst[3] = (double)m.q3;
        }
    }
}

__global__ void bump_counter(uint64_t* c, int n) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *c += (uint64_t)n;
}

__global__ void philox_kernel(const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t* out, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    u4 o = philox10({ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]}, k0, k1);
    out[4 * i] = o.x;
    out[4 * i + 1] = o.y;
    out[4 * i + 2] = o.z;
    out[4 * i + 3] = o.w;
}


// ---------------------------------------------------------------------------
// Batches of independent lattices.  A work item is (pass, lattice, tile);
// the lattices' tiles of one pass are concatenated (tile_prefix).
//
// batch_pass: one launch per pass index covers that pass of every member,
// kernel boundaries order the passes.
//
// batch_persistent: one launch for whole compound sweeps.  Blocks take items
// from a global counter in pass-major order; an item waits until every tile
// of the previous passes of its own lattice is done (per-lattice counters:
// relaxed polling with sleeps, then one agent-scope acquire fence; release
// by the finishing block), so members of different sizes advance
// independently with no grid-wide barrier.  Items are handed out in
// increasing order and depend only on smaller ones, so the smallest
// unfinished item can always run and the launch drains for any grid size.
// A bounded wait sets an abort flag that makes every later wait return at
// once, so even a broken invariant cannot keep the kernel alive.
// ---------------------------------------------------------------------------
template <class ST3, class ST2>
LAT_DEV void batch_site(const PassArgs& a, int kind, bool reunit, int64_t s) {
    if (a.group == 3) {
        if (kind == 0) {
            if (reunit) su3_site<ST3, 0, true, LAT_RNG_PHILOX_I>(a, s);
            else su3_site<ST3, 0, false, LAT_RNG_PHILOX_I>(a, s);
        } else {
            if (reunit) su3_site<ST3, 1, true, LAT_RNG_CONST_I>(a, s);
            else su3_site<ST3, 1, false, LAT_RNG_CONST_I>(a, s);
        }
    } else {
        if (kind == 0) {
            if (reunit) su2_site<ST2, 0, true, LAT_RNG_PHILOX_I>(a, s);
            else su2_site<ST2, 0, false, LAT_RNG_PHILOX_I>(a, s);
        } else {
            if (reunit) su2_site<ST2, 1, true, LAT_RNG_CONST_I>(a, s);
            else su2_site<ST2, 1, false, LAT_RNG_CONST_I>(a, s);
        }
    }
}

LAT_DEV int batch_member(const BatchArgs& b, int r) {
    int lo = 0, hi = b.nlat - 1;  // last member whose first tile is <= r
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (b.lats[mid].tile_prefix <= r) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// The same with the pass kind, reunitarisation and (overrelaxation)
// direction fixed at compile time, as the single-lattice passes are: the
// kernel then needs only the registers of its own kind.
template <class ST3, class ST2, int KIND, bool REUNIT, int MU>
LAT_DEV void batch_site_fixed(const PassArgs& a, int64_t s) {
    if (a.group == 3) {
        if constexpr (KIND == 0) su3_site<ST3, 0, REUNIT, LAT_RNG_PHILOX_I>(a, s);
        else su3_site<ST3, 1, REUNIT, LAT_RNG_CONST_I, MU>(a, s);
    } else {
        if constexpr (KIND == 0) su2_site<ST2, 0, REUNIT, LAT_RNG_PHILOX_I>(a, s);
        else su2_site<ST2, 1, REUNIT, LAT_RNG_CONST_I>(a, s);
    }
}

// Runs tile `tile` of member `m` for pass gp (counted from the launch start);
// KIND < 0: kind, reunitarisation and direction from gp at run time.
template <class ST3, class ST2, int KIND = -1, bool REUNIT = false, int MU = -1>
LAT_DEV void batch_tile(const BatchArgs& b, int m, int tile, int64_t gp) {
    const BatchLat& L = b.lats[m];
    const int sweep = (int)(gp / b.passes_per_sweep);
    const int pp = (int)(gp - (int64_t)sweep * b.passes_per_sweep);
    const int sw = pp >> 3;
    const int kind = sw < b.n_hb ? 0 : 1;
    const bool reunit = (sw == b.n_hb + b.n_or - 1);
    PassArgs a;
    a.g = L.g;
    a.links = L.links;
    a.mrg = nullptr;
    a.hb_count = L.hb_count;
    a.accept_log = nullptr;
    a.beta = L.beta;
    a.rng_const = L.rng_const;
    a.key0 = L.key0;
    a.key1 = L.key1;
    a.lat_id = L.lat_id;
    a.nhit = L.nhit;
    a.group = L.group;
    a.mu = (pp >> 1) & 3;
    a.parity = pp & 1;
    a.hb_offset = sweep * b.n_hb + (kind == 0 ? sw : 0);
    a.tile_order = 1;
    a.flux = L.flux;
    a.tshape[0] = a.tshape[1] = a.tshape[2] = a.tshape[3] = 0;
    a.tcount[0] = a.tcount[1] = a.tcount[2] = a.tcount[3] = 1;
    a.nyb = a.zslab = 1;
    a.lds_reserve = 0;
    a.reverse = 0;
    a.frozen = 0;
    const int64_t end = (int64_t)(tile + 1) * b.tile < L.g.vh ? (int64_t)(tile + 1) * b.tile : L.g.vh;
    for (int64_t s = (int64_t)tile * b.tile + threadIdx.x; s < end; s += blockDim.x) {
        if constexpr (KIND < 0) batch_site<ST3, ST2>(a, kind, reunit, s);
        else batch_site_fixed<ST3, ST2, KIND, REUNIT, MU>(a, s);
    }
}

// One launch per pass: work-group b takes the (member, tile) the host's map
// assigns it; the map gives each member to one XCD (work-group b runs on XCD
// b mod 8), so a member's neighbour links stay in that XCD's L2.
template <class ST3, class ST2, int KIND, bool REUNIT, int MU>
__global__ void __launch_bounds__(256) batch_pass(BatchArgs b, int64_t gp) {
    const BatchItem it = b.items[blockIdx.x];
    if (it.member < 0) return;
    batch_tile<ST3, ST2, KIND, REUNIT, MU>(b, it.member, it.tile, gp);
}

template <class ST3, class ST2>
__global__ void __launch_bounds__(256) batch_persistent(BatchArgs b) {
    __shared__ unsigned item_sh;
    const int64_t total = (int64_t)b.tiles_per_pass * b.passes_per_sweep * b.n_sweeps;
    for (;;) {
        if (threadIdx.x == 0) item_sh = atomicAdd(b.queue, 1u);
        __syncthreads();
        const int64_t item = item_sh;
        if (item >= total) return;  // uniform: every wave of the block leaves
        const int64_t gp = item / b.tiles_per_pass;
        const int r = (int)(item - gp * b.tiles_per_pass);
        const int m = batch_member(b, r);
        if (threadIdx.x == 0) {
            const unsigned need = (unsigned)gp * (unsigned)b.lats[m].ntiles;
            unsigned spins = 0;
            while (__hip_atomic_load(b.done + m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
                if (__hip_atomic_load(b.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
                __builtin_amdgcn_s_sleep(8);
                if (++spins > b.spin_limit) {
                    __hip_atomic_store(b.status, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
            }
            __atomic_thread_fence(__ATOMIC_ACQUIRE);
        }
        __syncthreads();
        batch_tile<ST3, ST2>(b, m, r - b.lats[m].tile_prefix, gp);
        // every wave's stores are complete before thread 0 releases the tile
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0) __hip_atomic_fetch_add(b.done + m, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ void batch_reset(BatchArgs b) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < b.nlat) b.done[i] = 0;
    if (i == 0) {
        *b.queue = 0;
        *b.status = 0;
    }
}

__global__ void batch_bump(BatchArgs b, uint64_t** counters, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < b.nlat) *counters[i] += (uint64_t)n;
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
LAT_HOST_DEV_INLINE unsigned pass_blocks(const PassArgs& a, int block) {
    if (a.tshape[0]) return (unsigned)a.tcount[0] * a.tcount[1] * a.tcount[2] * a.tcount[3];
    return (unsigned)((a.g.vh + block - 1) / block);
}

// Overrelaxation is specialised per direction; the heat bath takes the
// direction at run time (its straight-line form exceeds the register file).
template <class ST, int KIND, bool RE, int RNG>
hipError_t launch_su3(const PassArgs& a, int block, hipStream_t st) {
    const unsigned nb = pass_blocks(a, block);
    if constexpr (RNG != LAT_RNG_RANLUX_I) {
        if (a.stage_lds) {
            const size_t lds = (size_t)a.stage_lds;
            // per-direction overrelaxation only for FP32 12-real, as below
            constexpr bool PER_MU = KIND == 1 && std::is_same<ST, st_f32c12>::value;
            if constexpr (PER_MU) {
                switch (a.mu) {
                    case 0: hipLaunchKernelGGL((su3_pass_lq<ST, KIND, RE, RNG, 0>), dim3(nb), dim3(block), lds, st, a); break;
                    case 1: hipLaunchKernelGGL((su3_pass_lq<ST, KIND, RE, RNG, 1>), dim3(nb), dim3(block), lds, st, a); break;
                    case 2: hipLaunchKernelGGL((su3_pass_lq<ST, KIND, RE, RNG, 2>), dim3(nb), dim3(block), lds, st, a); break;
                    default: hipLaunchKernelGGL((su3_pass_lq<ST, KIND, RE, RNG, 3>), dim3(nb), dim3(block), lds, st, a); break;
                }
            } else {
                hipLaunchKernelGGL((su3_pass_lq<ST, KIND, RE, RNG, -1>), dim3(nb), dim3(block), lds, st, a);
            }
            return hipGetLastError();
        }
    }
    // Overrelaxation specialised per direction only for FP32 12-real: with
    // the two-row products (su3_site) the run-time-direction kernels of the
    // other forms are faster (MI355X, same run, 32^3x8 OR pass: FP64 18-real
    // 35.5 against 50.7 us, FP32 18-real 17.7 against 18.1 us, FP64 12-real
    // 25.8 against 26.8 us plain and 24.6 against 25.0 us staged; FP32
    // 12-real 13.46 against 13.24 us).  Heat baths always take it at run
    // time (their straight-line form spills).
    if constexpr (KIND == 1 && std::is_same<ST, st_f32c12>::value) {
        switch (a.mu) {
            case 0: hipLaunchKernelGGL((su3_pass<ST, KIND, RE, RNG, 0>), dim3(nb), dim3(block), a.lds_reserve, st, a); break;
            case 1: hipLaunchKernelGGL((su3_pass<ST, KIND, RE, RNG, 1>), dim3(nb), dim3(block), a.lds_reserve, st, a); break;
            case 2: hipLaunchKernelGGL((su3_pass<ST, KIND, RE, RNG, 2>), dim3(nb), dim3(block), a.lds_reserve, st, a); break;
            default: hipLaunchKernelGGL((su3_pass<ST, KIND, RE, RNG, 3>), dim3(nb), dim3(block), a.lds_reserve, st, a); break;
        }
    } else {
        hipLaunchKernelGGL((su3_pass<ST, KIND, RE, RNG, -1>), dim3(nb), dim3(block), a.lds_reserve, st, a);
    }
    return hipGetLastError();
}
template <class ST, int KIND, bool RE, int RNG>
hipError_t launch_su2(const PassArgs& a, int block, hipStream_t st) {
    const unsigned nb = pass_blocks(a, block);
    hipLaunchKernelGGL((su2_pass<ST, KIND, RE, RNG>), dim3(nb), dim3(block), a.lds_reserve, st, a);
    return hipGetLastError();
}

template <class ST, bool SU3, int K, bool R, int G>
hipError_t launch_one(const PassArgs& a, int block, hipStream_t st) {
    if constexpr (SU3) return launch_su3<ST, K, R, G>(a, block, st);
    else return launch_su2<ST, K, R, G>(a, block, st);
}

template <class ST, bool SU3>
hipError_t pass_dispatch(int kind, bool reunit, int rng, const PassArgs& a, int block, hipStream_t st) {
    if (kind == 1)
        return reunit ? launch_one<ST, SU3, 1, true, LAT_RNG_CONST_I>(a, block, st)
                      : launch_one<ST, SU3, 1, false, LAT_RNG_CONST_I>(a, block, st);
    switch (rng) {
        case LAT_RNG_MRG_I:
            return reunit ? launch_one<ST, SU3, 0, true, LAT_RNG_MRG_I>(a, block, st)
                          : launch_one<ST, SU3, 0, false, LAT_RNG_MRG_I>(a, block, st);
        case LAT_RNG_PHILOX_I:
            return reunit ? launch_one<ST, SU3, 0, true, LAT_RNG_PHILOX_I>(a, block, st)
                          : launch_one<ST, SU3, 0, false, LAT_RNG_PHILOX_I>(a, block, st);
        case LAT_RNG_RANLUX_I:
            return reunit ? launch_one<ST, SU3, 0, true, LAT_RNG_RANLUX_I>(a, block, st)
                          : launch_one<ST, SU3, 0, false, LAT_RNG_RANLUX_I>(a, block, st);
        default:
            return reunit ? launch_one<ST, SU3, 0, true, LAT_RNG_CONST_I>(a, block, st)
                          : launch_one<ST, SU3, 0, false, LAT_RNG_CONST_I>(a, block, st);
    }
}

}  // namespace

hipError_t lat_launch_pass(int group, int storage, int kind, bool reunit, int rng, const PassArgs& a, int block,
                           hipStream_t st) {
    if (group == 3) {
        switch (storage) {
            case LAT_ST_F64: return pass_dispatch<st_f64, true>(kind, reunit, rng, a, block, st);
            case LAT_ST_F32: return pass_dispatch<st_f32, true>(kind, reunit, rng, a, block, st);
            case LAT_ST_F64C12: return pass_dispatch<st_f64c12, true>(kind, reunit, rng, a, block, st);
            default: return pass_dispatch<st_f32c12, true>(kind, reunit, rng, a, block, st);
        }
    }
    if (storage == LAT_ST_F64) return pass_dispatch<sq_f64, false>(kind, reunit, rng, a, block, st);
    return pass_dispatch<sq_f32, false>(kind, reunit, rng, a, block, st);
}

template <class ST, bool SU3>
static hipError_t init_dispatch(int rng, const InitArgs& a, hipStream_t st) {
    dim3 grid((unsigned)((a.g.vh + 255) / 256), 2);
    switch (rng) {
        case LAT_RNG_MRG_I:
            if constexpr (SU3) hipLaunchKernelGGL((su3_init<ST, LAT_RNG_MRG_I>), grid, dim3(256), 0, st, a);
            else hipLaunchKernelGGL((su2_init<ST, LAT_RNG_MRG_I>), grid, dim3(256), 0, st, a);
            break;
        case LAT_RNG_PHILOX_I:
            if constexpr (SU3) hipLaunchKernelGGL((su3_init<ST, LAT_RNG_PHILOX_I>), grid, dim3(256), 0, st, a);
            else hipLaunchKernelGGL((su2_init<ST, LAT_RNG_PHILOX_I>), grid, dim3(256), 0, st, a);
            break;
        case LAT_RNG_RANLUX_I:
            if constexpr (SU3) hipLaunchKernelGGL((su3_init<ST, LAT_RNG_RANLUX_I>), grid, dim3(256), 0, st, a);
            else hipLaunchKernelGGL((su2_init<ST, LAT_RNG_RANLUX_I>), grid, dim3(256), 0, st, a);
            break;
        default:
            if constexpr (SU3) hipLaunchKernelGGL((su3_init<ST, LAT_RNG_CONST_I>), grid, dim3(256), 0, st, a);
            else hipLaunchKernelGGL((su2_init<ST, LAT_RNG_CONST_I>), grid, dim3(256), 0, st, a);
            break;
    }
    return hipGetLastError();
}

hipError_t lat_launch_init(int group, int storage, int rng, const InitArgs& a, hipStream_t st) {
    if (group == 3) {
        switch (storage) {
            case LAT_ST_F64: return init_dispatch<st_f64, true>(rng, a, st);
            case LAT_ST_F32: return init_dispatch<st_f32, true>(rng, a, st);
            case LAT_ST_F64C12: return init_dispatch<st_f64c12, true>(rng, a, st);
            default: return init_dispatch<st_f32c12, true>(rng, a, st);
        }
    }
    if (storage == LAT_ST_F64) return init_dispatch<sq_f64, false>(rng, a, st);
    return init_dispatch<sq_f32, false>(rng, a, st);
}

template <class ST, bool SU3>
static hipError_t meas_dispatch(const MeasArgs& a, double* out, uint32_t* slot, hipStream_t st) {
    dim3 gp((unsigned)(a.zslab ? 2 * a.nb_plaq : 16 * ((a.nb_plaq + 7) / 8)));
    dim3 gl((unsigned)a.nb_poly);
    if constexpr (SU3) hipLaunchKernelGGL((su3_plaq<ST>), gp, dim3(256), a.lds_reserve, st, a);
    else hipLaunchKernelGGL((su2_plaq<ST>), gp, dim3(256), a.lds_reserve, st, a);
    hipLaunchKernelGGL((lat_poly<ST>), gl, dim3(256), 0, st, a);
    hipLaunchKernelGGL(meas_final, dim3(1), dim3(256), 0, st, a, out, slot);
    return hipGetLastError();
}

hipError_t lat_launch_measure(int group, int storage, const MeasArgs& a, double* out, uint32_t* slot_counter,
                              hipStream_t st) {
    if (group == 3) {
        switch (storage) {
            case LAT_ST_F64: return meas_dispatch<st_f64, true>(a, out, slot_counter, st);
            case LAT_ST_F32: return meas_dispatch<st_f32, true>(a, out, slot_counter, st);
            case LAT_ST_F64C12: return meas_dispatch<st_f64c12, true>(a, out, slot_counter, st);
            default: return meas_dispatch<st_f32c12, true>(a, out, slot_counter, st);
        }
    }
    if (storage == LAT_ST_F64) return meas_dispatch<sq_f64, false>(a, out, slot_counter, st);
    return meas_dispatch<sq_f32, false>(a, out, slot_counter, st);
}

template <class ST, int NG>
static hipError_t conv_dispatch(bool to_dev, const LatGeom& g, double* canon, char* links, hipStream_t st) {
    dim3 grid((unsigned)((g.vh + 255) / 256), 2);
    if (to_dev) hipLaunchKernelGGL((to_device<ST, NG>), grid, dim3(256), 0, st, g, canon, links);
    else hipLaunchKernelGGL((to_canonical<ST, NG>), grid, dim3(256), 0, st, g, links, canon);
    return hipGetLastError();
}

hipError_t lat_launch_convert(int group, int storage, bool to_dev, const LatGeom& g, double* canon, char* links,
                              hipStream_t st) {
    if (group == 3) {
        switch (storage) {
            case LAT_ST_F64: return conv_dispatch<st_f64, 3>(to_dev, g, canon, links, st);
            case LAT_ST_F32: return conv_dispatch<st_f32, 3>(to_dev, g, canon, links, st);
            case LAT_ST_F64C12: return conv_dispatch<st_f64c12, 3>(to_dev, g, canon, links, st);
            default: return conv_dispatch<st_f32c12, 3>(to_dev, g, canon, links, st);
        }
    }
    if (storage == LAT_ST_F64) return conv_dispatch<sq_f64, 2>(to_dev, g, canon, links, st);
    return conv_dispatch<sq_f32, 2>(to_dev, g, canon, links, st);
}

hipError_t lat_launch_bump(uint64_t* counter, int n, hipStream_t st) {
    hipLaunchKernelGGL(bump_counter, dim3(1), dim3(64), 0, st, counter, n);
    return hipGetLastError();
}

hipError_t lat_launch_philox(const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t* out, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(philox_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ctr, k0, k1, out, n);
    return hipGetLastError();
}

template <class ST3, class ST2>
static void batch_launch_typed(const BatchArgs& b, int mode, int grid, int block, hipStream_t st) {
    if (mode == 1) {
        hipLaunchKernelGGL((batch_persistent<ST3, ST2>), dim3(grid), dim3(block), 0, st, b);
        return;
    }
    const int64_t npass = (int64_t)b.passes_per_sweep * b.n_sweeps;
    for (int64_t gp = 0; gp < npass; ++gp) {
        // pass gp of the launch: the same decomposition as batch_tile's
        const int pp = (int)(gp % b.passes_per_sweep);
        const int sw = pp >> 3, mu = (pp >> 1) & 3;
        const bool hb = sw < b.n_hb, re = (sw == b.n_hb + b.n_or - 1);
        const dim3 g(b.nitems), t(block);
        if (hb) {
            if (re) hipLaunchKernelGGL((batch_pass<ST3, ST2, 0, true, -1>), g, t, 0, st, b, gp);
            else hipLaunchKernelGGL((batch_pass<ST3, ST2, 0, false, -1>), g, t, 0, st, b, gp);
        } else if constexpr (!std::is_same<ST3, st_f32c12>::value) {
            // as for single lattices, overrelaxation takes the direction at
            // run time except in the FP32 12-real form (64-lattice scan:
            // FP64 4.49 -> 4.98, FP32 10.61 -> 11.38, FP64 12-real
            // 6.63 -> 6.98 1e9 link updates/s)
            if (re) hipLaunchKernelGGL((batch_pass<ST3, ST2, 1, true, -1>), g, t, 0, st, b, gp);
            else hipLaunchKernelGGL((batch_pass<ST3, ST2, 1, false, -1>), g, t, 0, st, b, gp);
        } else {
#define LAT_BATCH_OR(M)                                                                          \
    if (re) hipLaunchKernelGGL((batch_pass<ST3, ST2, 1, true, M>), g, t, 0, st, b, gp);          \
    else hipLaunchKernelGGL((batch_pass<ST3, ST2, 1, false, M>), g, t, 0, st, b, gp);
            switch (mu) {
                case 0: LAT_BATCH_OR(0) break;
                case 1: LAT_BATCH_OR(1) break;
                case 2: LAT_BATCH_OR(2) break;
                default: LAT_BATCH_OR(3) break;
            }
#undef LAT_BATCH_OR
        }
    }
}

hipError_t lat_launch_batch(int storage, int mode, const BatchArgs& b, uint64_t** counters, int grid, int block,
                            hipStream_t st) {
    const unsigned nb = (unsigned)((b.nlat + 255) / 256);
    if (mode == 1) hipLaunchKernelGGL(batch_reset, dim3(nb), dim3(256), 0, st, b);
    switch (storage) {
        case LAT_ST_F64: batch_launch_typed<st_f64, sq_f64>(b, mode, grid, block, st); break;
        case LAT_ST_F32: batch_launch_typed<st_f32, sq_f32>(b, mode, grid, block, st); break;
        case LAT_ST_F64C12: batch_launch_typed<st_f64c12, sq_f64>(b, mode, grid, block, st); break;
        default: batch_launch_typed<st_f32c12, sq_f32>(b, mode, grid, block, st); break;
    }
    if (b.n_hb > 0) hipLaunchKernelGGL(batch_bump, dim3(nb), dim3(256), 0, st, b, counters, b.n_hb * b.n_sweeps);
    return hipGetLastError();
}
