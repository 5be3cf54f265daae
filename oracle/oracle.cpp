/*
 * Plain FP64 CPU oracle for the checkerboard SU(2)/SU(3) Wilson-action
 * Monte Carlo.  TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check
 * and the CPU-baseline leg of the benchmark, never by the product path.
 *
 * What it follows (QCDGPU, arXiv:1310.7087):
 *   - SU(N) link fields stored per lattice site and direction (Sec. 3.3);
 *   - even/odd (checkerboard) update with a (pseudo-)heat bath (Sec. 3.3);
 *   - NHIT = 10 tries and reunitarisation in the SU(N) runs (Sec. 5);
 *   - hot (random) start (Sec. 5); per-run seed ("RANDSERIES", Sec. 3.4);
 *   - MRG32k3a as a multi-stream generator and a constant generator for
 *     debugging (Sec. 3.4);
 *   - an external magnetic-field flux as a run parameter (Sec. 1, 3.2).
 * The paper does not spell out the algorithms; the concrete textbook
 * choices (Kennedy-Pendleton SU(2) heat bath, Cabibbo-Marinari subgroups,
 * overrelaxation, Gram-Schmidt reunitarisation, the phase-twisted lambda_3
 * background, plaquette and Polyakov loop) are written out below step by
 * step in plain FP64 complex matrix arithmetic, with no blocking or fusion.
 * The oracle keeps the dynamical links U and multiplies by the fixed
 * background B on the fly; links are exported as W = U * B.
 */
#include "oracle.h"

#include <cmath>
#include <complex>
#include <random>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef std::complex<double> cplx;
static const double TWO_PI = 6.283185307179586476925286766559;

/* ------------------------------------------------------------------ */
/* N x N complex matrices, N = 2 or 3 (always stored 3x3).             */
/* ------------------------------------------------------------------ */
struct Mat {
    cplx a[3][3];
};

static Mat mat_zero() {
    Mat m;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) m.a[r][c] = 0.0;
    return m;
}
static Mat mat_identity(int n) {
    Mat m = mat_zero();
    for (int r = 0; r < n; ++r) m.a[r][r] = 1.0;
    return m;
}
static Mat mat_mul(int n, const Mat& x, const Mat& y) {
    Mat m = mat_zero();
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) {
            cplx s = 0.0;
            for (int k = 0; k < n; ++k) s += x.a[r][k] * y.a[k][c];
            m.a[r][c] = s;
        }
    return m;
}
static Mat mat_dag(int n, const Mat& x) {
    Mat m = mat_zero();
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) m.a[r][c] = std::conj(x.a[c][r]);
    return m;
}
static Mat mat_add(int n, const Mat& x, const Mat& y) {
    Mat m = mat_zero();
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) m.a[r][c] = x.a[r][c] + y.a[r][c];
    return m;
}
static double re_trace(int n, const Mat& x) {
    double s = 0.0;
    for (int r = 0; r < n; ++r) s += x.a[r][r].real();
    return s;
}
static cplx trace(int n, const Mat& x) {
    cplx s = 0.0;
    for (int r = 0; r < n; ++r) s += x.a[r][r];
    return s;
}

/* Quaternion q = (q0,q1,q2,q3) <-> 2x2 matrix q0*1 + i(q1 s1 + q2 s2 + q3 s3). */
static void quat_to_2x2(const double q[4], cplx m[2][2]) {
    m[0][0] = cplx(q[0], q[3]);
    m[0][1] = cplx(q[2], q[1]);
    m[1][0] = cplx(-q[2], q[1]);
    m[1][1] = cplx(q[0], -q[3]);
}
/* SU(2) projection of a general complex 2x2 block (w11,w12;w21,w22):
 * the quaternion part, which alone contributes to Re Tr(r w) for r in SU(2). */
static void project_2x2(const cplx& w11, const cplx& w12, const cplx& w21,
                        const cplx& w22, double q[4]) {
    q[0] = 0.5 * (w11 + w22).real();
    q[1] = 0.5 * (w12 + w21).imag();
    q[2] = 0.5 * (w12 - w21).real();
    q[3] = 0.5 * (w11 - w22).imag();
}

/* Gram-Schmidt reunitarisation: normalise row 1, orthogonalise and
 * normalise row 2, row 3 = conj(row1 x row2) so that det = 1.  For SU(2)
 * the quaternion part is normalised. */
static Mat reunitarise(int n, const Mat& x) {
    if (n == 2) {
        double q[4];
        project_2x2(x.a[0][0], x.a[0][1], x.a[1][0], x.a[1][1], q);
        double nn = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        for (int k = 0; k < 4; ++k) q[k] /= nn;
        cplx m[2][2];
        quat_to_2x2(q, m);
        Mat r = mat_zero();
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) r.a[a][b] = m[a][b];
        return r;
    }
    Mat r = mat_zero();
    cplx r1[3], r2[3];
    double n1 = 0.0;
    for (int c = 0; c < 3; ++c) n1 += std::norm(x.a[0][c]);
    n1 = std::sqrt(n1);
    for (int c = 0; c < 3; ++c) r1[c] = x.a[0][c] / n1;
    cplx dot = 0.0;  // r1^dagger . row2
    for (int c = 0; c < 3; ++c) dot += std::conj(r1[c]) * x.a[1][c];
    for (int c = 0; c < 3; ++c) r2[c] = x.a[1][c] - dot * r1[c];
    double n2 = 0.0;
    for (int c = 0; c < 3; ++c) n2 += std::norm(r2[c]);
    n2 = std::sqrt(n2);
    for (int c = 0; c < 3; ++c) r2[c] /= n2;
    for (int c = 0; c < 3; ++c) {
        r.a[0][c] = r1[c];
        r.a[1][c] = r2[c];
    }
    r.a[2][0] = std::conj(r1[1] * r2[2] - r1[2] * r2[1]);
    r.a[2][1] = std::conj(r1[2] * r2[0] - r1[0] * r2[2]);
    r.a[2][2] = std::conj(r1[0] * r2[1] - r1[1] * r2[0]);
    return r;
}

/* ------------------------------------------------------------------ */
/* Random numbers                                                      */
/* ------------------------------------------------------------------ */
double orc_uniform24(uint32_t w) {
    /* 24 high bits, centred in their cell: exact in FP32 and FP64, in (0,1). */
    return ((double)(w >> 8) + 0.5) * (1.0 / 16777216.0);
}

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two
 * 32x32->64 multiplies with the key bumped by the Weyl constants. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* MRG32k3a (L'Ecuyer 1999): two order-3 recursions
 *   x1[n] = (1403580 x1[n-2] - 810728 x1[n-3]) mod m1,
 *   x2[n] = (527612 x2[n-1] - 1370589 x2[n-3]) mod m2,
 * output z = (x1[n] - x2[n]) mod m1 taken in [1, m1]. */
static const uint64_t MRG_M1 = 4294967087ull;
static const uint64_t MRG_M2 = 4294944443ull;

uint32_t orc_mrg_next(uint32_t st[6]) {
    uint64_t x1 = ((unsigned __int128)1403580u * st[1] +
                   (unsigned __int128)(MRG_M1 - 810728u) * st[0]) % MRG_M1;
    uint64_t x2 = ((unsigned __int128)527612u * st[5] +
                   (unsigned __int128)(MRG_M2 - 1370589u) * st[3]) % MRG_M2;
    st[0] = st[1]; st[1] = st[2]; st[2] = (uint32_t)x1;
    st[3] = st[4]; st[4] = st[5]; st[5] = (uint32_t)x2;
    return x1 > x2 ? (uint32_t)(x1 - x2) : (uint32_t)(x1 + MRG_M1 - x2);
}

/* 3x3 transition matrices acting on column (x[n-3], x[n-2], x[n-1]). */
typedef uint64_t M33[3][3];
static void m33_mul(const M33 a, const M33 b, uint64_t m, M33 out) {
    M33 t;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            unsigned __int128 s = 0;
            for (int k = 0; k < 3; ++k) s += (unsigned __int128)a[r][k] * b[k][c] % m;
            t[r][c] = (uint64_t)(s % m);
        }
    std::memcpy(out, t, sizeof(M33));
}
static void m33_vec(const M33 a, const uint32_t* v, uint64_t m, uint32_t* out) {
    uint64_t t[3];
    for (int r = 0; r < 3; ++r) {
        unsigned __int128 s = 0;
        for (int k = 0; k < 3; ++k) s += (unsigned __int128)a[r][k] * v[k] % m;
        t[r] = (uint64_t)(s % m);
    }
    for (int r = 0; r < 3; ++r) out[r] = (uint32_t)t[r];
}
static void mrg_base(M33 a1, M33 a2) {
    const M33 b1 = {{0, 1, 0}, {0, 0, 1}, {MRG_M1 - 810728u, 1403580u, 0}};
    const M33 b2 = {{0, 1, 0}, {0, 0, 1}, {MRG_M2 - 1370589u, 0, 527612u}};
    std::memcpy(a1, b1, sizeof(M33));
    std::memcpy(a2, b2, sizeof(M33));
}
static void mrg_pow2(int e, M33 a1, M33 a2) {
    mrg_base(a1, a2);
    for (int k = 0; k < e; ++k) {
        m33_mul(a1, a1, MRG_M1, a1);
        m33_mul(a2, a2, MRG_M2, a2);
    }
}
void orc_mrg_advance_pow2(uint32_t st[6], int e) {
    M33 a1, a2;
    mrg_pow2(e, a1, a2);
    m33_vec(a1, st, MRG_M1, st);
    m33_vec(a2, st + 3, MRG_M2, st + 3);
}
int orc_mrg_site_state(uint64_t seed, uint64_t site, uint32_t st[6]) {
    if (seed < 1 || seed >= MRG_M2) return -1;
    for (int k = 0; k < 6; ++k) st[k] = (uint32_t)seed;
    /* jump = A^(2^127); apply jump^site by binary powering */
    M33 j1, j2;
    mrg_pow2(127, j1, j2);
    uint64_t e = site;
    while (e) {
        if (e & 1) {
            m33_vec(j1, st, MRG_M1, st);
            m33_vec(j2, st + 3, MRG_M2, st + 3);
        }
        m33_mul(j1, j1, MRG_M1, j1);
        m33_mul(j2, j2, MRG_M2, j2);
        e >>= 1;
    }
    return 0;
}

/* Where the uniforms of one link update come from. */
struct Draws {
    virtual void try4(int g, int t, double u[4]) = 0;  // R1..R4 of try t
    virtual void dir2(int g, double u[2]) = 0;         // R5, R6
    virtual ~Draws() {}
};
struct PhiloxDraws : Draws {
    uint32_t key[2], site, lat, word2;
    int nhit;
    void try4(int g, int t, double u[4]) override {
        uint32_t c[4] = {site, lat, word2, (uint32_t)(g * (nhit + 1) + t)}, o[4];
        orc_philox4x32_10(c, key, o);
        for (int k = 0; k < 4; ++k) u[k] = orc_uniform24(o[k]);
    }
    void dir2(int g, double u[2]) override {
        uint32_t c[4] = {site, lat, word2, (uint32_t)(g * (nhit + 1) + nhit)}, o[4];
        orc_philox4x32_10(c, key, o);
        u[0] = orc_uniform24(o[0]);
        u[1] = orc_uniform24(o[1]);
    }
};
struct MrgDraws : Draws {
    uint32_t* st;
    void try4(int, int, double u[4]) override {
        for (int k = 0; k < 4; ++k) u[k] = orc_uniform24(orc_mrg_next(st));
    }
    void dir2(int, double u[2]) override {
        for (int k = 0; k < 2; ++k) u[k] = orc_uniform24(orc_mrg_next(st));
    }
};
/* RANLUX, luxury level 3 (Luscher 1994; James 1994): the subtract-with-
 * borrow generator x_n = x_{n-10} - x_{n-24} - c mod 2^24 of which, in every
 * block of p = 223 consecutive outputs, the first r = 24 are used and the
 * rest discarded.  The C++ standard library defines both pieces
 * (subtract_with_carry_engine<24, 10, 24> is ranlux24_base, and
 * discard_block_engine takes p and r), so the oracle composes them. */
typedef std::discard_block_engine<std::ranlux24_base, 223, 24> Ranlux3;
/* Reading of the draw rule for RANLUX: every link update (and every link's
 * hot-start draw) begins a new block of its site's stream; what the
 * previous update left of its block is skipped.  A site's stream is seeded
 * with 1 + (seed + 1000003 (i + 2654435761 lattice_id)) mod 2147483561. */
struct RanluxSite {
    Ranlux3 eng;
    int used = 0;         // values drawn from the current block
    bool claimed = false; // a block has been begun
    void begin_update() {
        if (claimed) eng.discard(24 - used);
        used = 0;
        claimed = true;
    }
    double next() {
        if (used == 24) used = 0;  // an update that needs more runs into the next block
        ++used;
        return orc_uniform24((uint32_t)eng() << 8);
    }
};
struct RanluxDraws : Draws {
    RanluxSite* st;
    void try4(int, int, double u[4]) override {
        for (int k = 0; k < 4; ++k) u[k] = st->next();
    }
    void dir2(int, double u[2]) override {
        for (int k = 0; k < 2; ++k) u[k] = st->next();
    }
};
uint32_t ranlux_site_seed(uint64_t seed, int64_t i, uint32_t lattice_id) {
    const uint64_t M = 2147483561ull;
    const uint64_t j = ((uint64_t)i + 2654435761ull * (uint64_t)lattice_id) % M;
    return (uint32_t)(1 + ((seed % M) + 1000003ull * j) % M);
}

struct ConstDraws : Draws {
    double c;
    void try4(int, int, double u[4]) override { u[0] = u[1] = u[2] = u[3] = c; }
    void dir2(int, double u[2]) override { u[0] = u[1] = c; }
};
struct ArrayDraws : Draws {
    const double* u;
    int pos = 0;
    void try4(int, int, double o[4]) override {
        for (int k = 0; k < 4; ++k) o[k] = u[pos++];
    }
    void dir2(int, double o[2]) override {
        for (int k = 0; k < 2; ++k) o[k] = u[pos++];
    }
};

/* ------------------------------------------------------------------ */
/* Kennedy-Pendleton SU(2) heat bath: sample a0 with density            */
/* sqrt(1-a0^2) exp(alpha a0) via lambda^2 ~ lambda^2 exp(-2 alpha      */
/* lambda^2) and acceptance sqrt(1-lambda^2); a0 = 1 - 2 lambda^2;      */
/* direction of (a1,a2,a3) uniform on the sphere.                       */
/* ------------------------------------------------------------------ */
static int kp_draw(double alpha, int nhit, Draws& d, int g, double x[4]) {
    for (int t = 0; t < nhit; ++t) {
        double R[4];
        d.try4(g, t, R);
        double c = std::cos(TWO_PI * R[1]);
        double lam2 = -(std::log(R[0]) + c * c * std::log(R[2])) / (2.0 * alpha);
        if (R[3] * R[3] <= 1.0 - lam2) {
            double D[2];
            d.dir2(g, D);
            double a0 = 1.0 - 2.0 * lam2;
            double s = 2.0 * std::sqrt(lam2 * (1.0 - lam2));
            double ct = 2.0 * D[0] - 1.0;
            double st = std::sqrt(1.0 - ct * ct);
            double ph = TWO_PI * D[1];
            x[0] = a0;
            x[1] = s * st * std::cos(ph);
            x[2] = s * st * std::sin(ph);
            x[3] = s * ct;
            return t;
        }
    }
    x[0] = 1.0; x[1] = x[2] = x[3] = 0.0;
    return -1;
}

int orc_kp_sample(double alpha, int nhit, const double* u, double x[4], int* used) {
    ArrayDraws d;
    d.u = u;
    int t = kp_draw(alpha, nhit, d, 0, x);
    if (used) *used = d.pos;
    return t;
}

/* SU(2) subgroups of SU(N) used in the pseudo-heat bath (Cabibbo-Marinari):
 * row/column pairs, in update order. */
static int n_subgroups(int n) { return n == 3 ? 3 : 1; }
static void subgroup(int g, int& a, int& b) {
    static const int P[3][2] = {{0, 1}, {1, 2}, {0, 2}};
    a = P[g][0];
    b = P[g][1];
}

/* Update link U with M = W*A (W = U*B the effective link, A its staple).
 * kind 0: heat bath; kind 1: overrelaxation.  For each subgroup the SU(2)
 * element r multiplies from the left: U <- R U and M <- R M.
 * accept[g] receives the accepted try (or -1) for heat-bath updates. */
static Mat update_with(int n, double beta, int nhit, int kind, Mat U, Mat M,
                       Draws& d, int8_t* accept) {
    for (int g = 0; g < n_subgroups(n); ++g) {
        int a, b;
        subgroup(g, a, b);
        double q[4];
        project_2x2(M.a[a][a], M.a[a][b], M.a[b][a], M.a[b][b], q);
        double k = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        double v[4];
        cplx rm[2][2];
        if (kind == 0) {
            double alpha = 2.0 * beta * k / n;
            if (accept) accept[g] = -1;
            if (!(alpha >= 1e-12)) continue;  // no coupling to the staple: leave unchanged
            double x[4];
            int t = kp_draw(alpha, nhit, d, g, x);
            if (accept) accept[g] = (int8_t)t;
            if (t < 0) continue;  // all tries rejected: subgroup unchanged
            for (int c = 0; c < 4; ++c) v[c] = q[c] / k;
            cplx X[2][2], V[2][2];
            quat_to_2x2(x, X);
            quat_to_2x2(v, V);
            /* r = X V^dagger */
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j)
                    rm[i][j] = X[i][0] * std::conj(V[j][0]) + X[i][1] * std::conj(V[j][1]);
        } else {
            if (!(k > 0.0)) continue;
            for (int c = 0; c < 4; ++c) v[c] = q[c] / k;
            cplx V[2][2], Vd[2][2];
            quat_to_2x2(v, V);
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j) Vd[i][j] = std::conj(V[j][i]);
            /* r = (V^dagger)^2: reflects r*v to its inverse, keeping Re Tr(R M) */
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j) rm[i][j] = Vd[i][0] * Vd[0][j] + Vd[i][1] * Vd[1][j];
        }
        Mat R = mat_identity(n);
        R.a[a][a] = rm[0][0];
        R.a[a][b] = rm[0][1];
        R.a[b][a] = rm[1][0];
        R.a[b][b] = rm[1][1];
        U = mat_mul(n, R, U);
        M = mat_mul(n, R, M);
    }
    return U;
}

/* ------------------------------------------------------------------ */
/* Lattice                                                             */
/* ------------------------------------------------------------------ */
struct orc_lattice {
    int n;          // gauge group SU(n)
    int d[4];       // Nx, Ny, Nz, Nt
    int64_t V;
    double beta;
    int flux;
    int rng;
    double rng_const;
    uint64_t seed;
    int nhit;
    uint32_t lat_id;
    int frozen;          // 1: spatial links of the slice t = 0 held at U = 1
    uint64_t hb_sweeps;  // heat-bath sweeps done so far (Philox counter word)
    std::vector<Mat> U;  // U-frame links, index i*4+mu
    std::vector<uint32_t> mrg;  // 6 words per site
    std::vector<RanluxSite> ranlux;  // one stream per site
    bool log_accept = false;
    std::vector<int8_t> accept_log;  // [k][mu][i][g]
};

static void coords(const orc_lattice* L, int64_t i, int x[4]) {
    for (int m = 0; m < 4; ++m) {
        x[m] = (int)(i % L->d[m]);
        i /= L->d[m];
    }
}
static int64_t index_of(const orc_lattice* L, const int x[4]) {
    int64_t i = 0;
    for (int m = 3; m >= 0; --m) i = i * L->d[m] + ((x[m] % L->d[m]) + L->d[m]) % L->d[m];
    return i;
}
static int64_t shift(const orc_lattice* L, int64_t i, int mu, int step) {
    int x[4];
    coords(L, i, x);
    x[mu] += step;
    return index_of(L, x);
}

/* Background field: diagonal exp(i theta T), T = diag(1,-1[,0]);
 * flux phi = 2 pi n / (Nx Ny) through every x-y plaquette:
 * B_y(x) = exp(i phi x1 T); B_x(x) = exp(-i phi Nx x2 T) at x1 = Nx-1, else 1. */
static double bg_theta(const orc_lattice* L, int64_t i, int mu) {
    if (L->flux == 0 || mu > 1) return 0.0;
    int x[4];
    coords(L, i, x);
    double phi = TWO_PI * (double)L->flux / (double)(L->d[0] * L->d[1]);
    if (mu == 1) return phi * (double)x[0];
    if (x[0] == L->d[0] - 1) return -phi * (double)(L->d[0] * x[1]);
    return 0.0;
}
static Mat background(const orc_lattice* L, int64_t i, int mu) {
    Mat b = mat_identity(L->n);
    double th = bg_theta(L, i, mu);
    if (th != 0.0) {
        b.a[0][0] = cplx(std::cos(th), std::sin(th));
        b.a[1][1] = cplx(std::cos(th), -std::sin(th));
    }
    return b;
}
/* Effective link W = U B. */
static Mat wlink(const orc_lattice* L, int64_t i, int mu) {
    return mat_mul(L->n, L->U[i * 4 + mu], background(L, i, mu));
}

/* Staple: sum over nu != mu (ascending) of the forward term
 * W_nu(x+mu) W_mu(x+nu)^+ W_nu(x)^+ and then the backward term
 * W_nu(x+mu-nu)^+ W_mu(x-nu)^+ W_nu(x-nu). */
static Mat staple(const orc_lattice* L, int64_t i, int mu) {
    int n = L->n;
    Mat A = mat_zero();
    int64_t xp = shift(L, i, mu, +1);
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        int64_t xpn = shift(L, i, nu, +1);
        int64_t xmn = shift(L, i, nu, -1);
        int64_t xpmn = shift(L, xp, nu, -1);
        Mat f = mat_mul(n, mat_mul(n, wlink(L, xp, nu), mat_dag(n, wlink(L, xpn, mu))),
                        mat_dag(n, wlink(L, i, nu)));
        A = mat_add(n, A, f);
        Mat bk = mat_mul(n, mat_mul(n, mat_dag(n, wlink(L, xpmn, nu)), mat_dag(n, wlink(L, xmn, mu))),
                         wlink(L, xmn, nu));
        A = mat_add(n, A, bk);
    }
    return A;
}

void orc_staple(const orc_lattice* L, int64_t i, int mu, double* out) {
    Mat A = staple(L, i, mu);
    for (int r = 0; r < L->n; ++r)
        for (int c = 0; c < L->n; ++c) {
            out[2 * (r * L->n + c)] = A.a[r][c].real();
            out[2 * (r * L->n + c) + 1] = A.a[r][c].imag();
        }
}

/* Haar-random SU(N) from uniforms via Box-Muller Gaussians:
 * SU(2): normalised 4-vector of Gaussians; SU(3): two rows of complex
 * Gaussians, Gram-Schmidt, row 3 = conj(row1 x row2). */
static void box_muller(double u1, double u2, double& g1, double& g2) {
    double r = std::sqrt(-2.0 * std::log(u1));
    g1 = r * std::cos(TWO_PI * u2);
    g2 = r * std::sin(TWO_PI * u2);
}
static Mat haar(int n, const double* u) {
    if (n == 2) {
        double g[4];
        box_muller(u[0], u[1], g[0], g[1]);
        box_muller(u[2], u[3], g[2], g[3]);
        double nn = std::sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2] + g[3] * g[3]);
        double q[4] = {g[0] / nn, g[1] / nn, g[2] / nn, g[3] / nn};
        cplx m[2][2];
        quat_to_2x2(q, m);
        Mat r = mat_zero();
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) r.a[a][b] = m[a][b];
        return r;
    }
    Mat G = mat_zero();
    for (int row = 0; row < 2; ++row)
        for (int c = 0; c < 3; ++c) {
            double re, im;
            box_muller(u[6 * row + 2 * c], u[6 * row + 2 * c + 1], re, im);
            G.a[row][c] = cplx(re, im);
        }
    return reunitarise(3, G);
}

static int ncomp(int n) { return n == 3 ? 18 : 4; }

static void to_canonical(int n, const Mat& W, double* out) {
    if (n == 2) {
        project_2x2(W.a[0][0], W.a[0][1], W.a[1][0], W.a[1][1], out);
        return;
    }
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            out[2 * (3 * r + c)] = W.a[r][c].real();
            out[2 * (3 * r + c) + 1] = W.a[r][c].imag();
        }
}
static Mat from_canonical(int n, const double* in) {
    Mat W = mat_zero();
    if (n == 2) {
        cplx m[2][2];
        quat_to_2x2(in, m);
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) W.a[a][b] = m[a][b];
        return W;
    }
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) W.a[r][c] = cplx(in[2 * (3 * r + c)], in[2 * (3 * r + c) + 1]);
    return W;
}

orc_lattice* orc_create(int group, int nx, int ny, int nz, int nt, double beta, int flux,
                        int rng, double rng_const, uint64_t seed, int nhit, uint32_t lattice_id,
                        int start, int frozen) {
    int dims[4] = {nx, ny, nz, nt};
    if (group != 2 && group != 3) return nullptr;
    for (int m = 0; m < 4; ++m)
        if (dims[m] < 2 || dims[m] % 2) return nullptr;
    if (!(beta >= 0.0) || nhit < 1 || nhit > 127) return nullptr;
    if (rng < 0 || rng > 3) return nullptr;
    if (rng == ORC_RNG_MRG32K3A && (seed < 1 || seed >= MRG_M2)) return nullptr;
    if (frozen != 0 && frozen != 1) return nullptr;
    // constant uniforms would make the two complex-Gaussian rows of an SU(3)
    // Haar start equal (Gram-Schmidt then has nothing to orthonormalise)
    if (group == 3 && rng == ORC_RNG_CONST && start == ORC_HOT) return nullptr;
    orc_lattice* L = new orc_lattice();
    L->frozen = frozen;
    L->n = group;
    for (int m = 0; m < 4; ++m) L->d[m] = dims[m];
    L->V = (int64_t)nx * ny * nz * nt;
    L->beta = beta;
    L->flux = flux;
    L->rng = rng;
    L->rng_const = rng_const;
    L->seed = seed;
    L->nhit = nhit;
    L->lat_id = lattice_id;
    L->hb_sweeps = 0;
    L->U.assign(L->V * 4, mat_identity(group));
    if (rng == ORC_RNG_MRG32K3A) {
        L->mrg.resize(L->V * 6);
        uint32_t st[6];
        orc_mrg_site_state(seed, 0, st);
        M33 j1, j2;
        mrg_pow2(127, j1, j2);
        for (int64_t i = 0; i < L->V; ++i) {
            std::memcpy(&L->mrg[6 * i], st, sizeof(st));
            m33_vec(j1, st, MRG_M1, st);
            m33_vec(j2, st + 3, MRG_M2, st + 3);
        }
    }
    if (rng == ORC_RNG_RANLUX) {
        L->ranlux.resize(L->V);
        for (int64_t i = 0; i < L->V; ++i) L->ranlux[i].eng.seed(ranlux_site_seed(seed, i, lattice_id));
    }
    if (start == ORC_HOT) {
        int nu = group == 3 ? 12 : 4;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < L->V; ++i) {
            for (int mu = 0; mu < 4; ++mu) {
                double u[12];
                if (rng == ORC_RNG_PHILOX) {
                    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
                    for (int j = 0; j < nu / 4; ++j) {
                        uint32_t c[4] = {(uint32_t)i, lattice_id, 0xFFFFFFFFu, (uint32_t)(4 * mu + j)}, o[4];
                        orc_philox4x32_10(c, key, o);
                        for (int k = 0; k < 4; ++k) u[4 * j + k] = orc_uniform24(o[k]);
                    }
                } else if (rng == ORC_RNG_MRG32K3A) {
                    for (int k = 0; k < nu; ++k) u[k] = orc_uniform24(orc_mrg_next(&L->mrg[6 * i]));
                } else if (rng == ORC_RNG_RANLUX) {
                    L->ranlux[i].begin_update();
                    for (int k = 0; k < nu; ++k) u[k] = L->ranlux[i].next();
                } else {
                    for (int k = 0; k < nu; ++k) u[k] = rng_const;
                }
                L->U[i * 4 + mu] = haar(group, u);
            }
        }
    }
    // Frozen external field: the spatial links of the slice t = 0 are the
    // background itself, W = B, i.e. U = 1 (their hot-start draws are made
    // and discarded, so every other link sees the same random numbers).
    if (frozen) {
        for (int64_t i = 0; i < L->V; ++i) {
            int x[4];
            coords(L, i, x);
            if (x[3] == 0)
                for (int mu = 0; mu < 3; ++mu) L->U[i * 4 + mu] = mat_identity(group);
        }
    }
    return L;
}

void orc_destroy(orc_lattice* L) { delete L; }

void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
int orc_get_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* One checkerboard pass: all links U_mu(x) with parity(x) = p. */
static void pass(orc_lattice* L, int mu, int p, int kind, bool reunit, int hb_index) {
    const int n = L->n;
    std::vector<int64_t> sites;
    sites.reserve(L->V / 2);
    for (int64_t i = 0; i < L->V; ++i) {
        int x[4];
        coords(L, i, x);
        if (L->frozen && mu < 3 && x[3] == 0) continue;  // held at the background, no draws
        if (((x[0] + x[1] + x[2] + x[3]) & 1) == p) sites.push_back(i);
    }
    const int64_t ns = (int64_t)sites.size();
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < ns; ++s) {
        int64_t i = sites[s];
        Mat A = staple(L, i, mu);
        Mat M = mat_mul(n, wlink(L, i, mu), A);
        PhiloxDraws pd;
        MrgDraws md;
        RanluxDraws rd;
        ConstDraws cd;
        Draws* d;
        if (L->rng == ORC_RNG_PHILOX) {
            pd.key[0] = (uint32_t)L->seed;
            pd.key[1] = (uint32_t)(L->seed >> 32);
            pd.site = (uint32_t)i;
            pd.lat = L->lat_id;
            pd.word2 = (uint32_t)(4 * L->hb_sweeps + mu);
            pd.nhit = L->nhit;
            d = &pd;
        } else if (L->rng == ORC_RNG_MRG32K3A) {
            md.st = &L->mrg[6 * i];
            d = &md;
        } else if (L->rng == ORC_RNG_RANLUX) {
            rd.st = &L->ranlux[i];
            if (kind == 0) rd.st->begin_update();
            d = &rd;
        } else {
            cd.c = L->rng_const;
            d = &cd;
        }
        int8_t* acc = nullptr;
        if (kind == 0 && L->log_accept)
            acc = &L->accept_log[(((int64_t)hb_index * 4 + mu) * L->V + i) * 3];
        Mat Unew = update_with(n, L->beta, L->nhit, kind, L->U[i * 4 + mu], M, *d, acc);
        if (reunit) Unew = reunitarise(n, Unew);
        L->U[i * 4 + mu] = Unew;
    }
}

void orc_sweep(orc_lattice* L, int n_hb, int n_or) {
    if (n_hb < 0 || n_or < 0) return;
    int total = n_hb + n_or;
    if (L->log_accept) L->accept_log.assign((size_t)n_hb * 4 * L->V * 3, (int8_t)-1);
    for (int s = 0; s < total; ++s) {
        int kind = s < n_hb ? 0 : 1;
        bool last = (s == total - 1);
        for (int mu = 0; mu < 4; ++mu)
            for (int p = 0; p < 2; ++p) pass(L, mu, p, kind, last, s);
        if (kind == 0) L->hb_sweeps++;
    }
}

/* Neumaier compensated sum of a vector, in index order. */
static double neumaier(const std::vector<double>& v) {
    double s = 0.0, c = 0.0;
    for (double x : v) {
        double t = s + x;
        if (std::fabs(s) >= std::fabs(x))
            c += (s - t) + x;
        else
            c += (x - t) + s;
        s = t;
    }
    return s + c;
}

/* Plaquette P_{mu nu}(x) = W_mu(x) W_nu(x+mu) W_mu(x+nu)^+ W_nu(x)^+;
 * P_s averages (1/N) Re Tr over the three spatial planes, P_t over the three
 * planes containing t, P over all six.  Polyakov loop
 * L(x) = (1/N) Tr prod_{t=0}^{Nt-1} W_t(x,t), averaged over spatial sites. */
void orc_measure(const orc_lattice* L, double plaq[3], double poly[2]) {
    const int n = L->n;
    std::vector<double> ps(L->V), pt(L->V);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < L->V; ++i) {
        double s_s = 0.0, s_t = 0.0;
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu) {
                int64_t xpm = shift(L, i, mu, +1), xpn = shift(L, i, nu, +1);
                Mat P = mat_mul(n, mat_mul(n, mat_mul(n, wlink(L, i, mu), wlink(L, xpm, nu)),
                                           mat_dag(n, wlink(L, xpn, mu))),
                                mat_dag(n, wlink(L, i, nu)));
                double v = re_trace(n, P) / n;
                if (nu == 3)
                    s_t += v;
                else
                    s_s += v;
            }
        ps[i] = s_s;
        pt[i] = s_t;
    }
    double Ps = neumaier(ps) / (3.0 * L->V);
    double Pt = neumaier(pt) / (3.0 * L->V);
    plaq[0] = 0.5 * (Ps + Pt);
    plaq[1] = Ps;
    plaq[2] = Pt;
    int64_t Vs = L->V / L->d[3];
    std::vector<double> lr(Vs), li(Vs);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < Vs; ++s) {
        Mat P = mat_identity(n);
        for (int t = 0; t < L->d[3]; ++t) P = mat_mul(n, P, wlink(L, s + Vs * t, 3));
        cplx tr = trace(n, P) / (double)n;
        lr[s] = tr.real();
        li[s] = tr.imag();
    }
    poly[0] = neumaier(lr) / (double)Vs;
    poly[1] = neumaier(li) / (double)Vs;
}

void orc_get_links(const orc_lattice* L, double* out) {
    const int nc = ncomp(L->n);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < L->V; ++i)
        for (int mu = 0; mu < 4; ++mu) to_canonical(L->n, wlink(L, i, mu), out + (i * 4 + mu) * nc);
}

void orc_set_links(orc_lattice* L, const double* in) {
    const int nc = ncomp(L->n);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < L->V; ++i)
        for (int mu = 0; mu < 4; ++mu) {
            Mat W = from_canonical(L->n, in + (i * 4 + mu) * nc);
            L->U[i * 4 + mu] = mat_mul(L->n, W, mat_dag(L->n, background(L, i, mu)));
        }
}

uint64_t orc_hb_sweeps(const orc_lattice* L) { return L->hb_sweeps; }

void orc_ranlux_raw(uint32_t seed, int n, int luxury_blocks, uint32_t* out) {
    if (luxury_blocks) {
        Ranlux3 e(seed);
        for (int k = 0; k < n; ++k) out[k] = (uint32_t)e();
    } else {
        std::ranlux24_base e(seed);
        for (int k = 0; k < n; ++k) out[k] = (uint32_t)e();
    }
}

void orc_ranlux_standard_values(uint32_t out[2]) {
    std::ranlux24_base a;
    std::ranlux24 b;
    a.discard(9999);
    b.discard(9999);
    out[0] = (uint32_t)a();
    out[1] = (uint32_t)b();
}

uint32_t orc_ranlux_site_seed(uint64_t seed, int64_t i, uint32_t lattice_id) {
    return ranlux_site_seed(seed, i, lattice_id);
}

int orc_get_mrg_states(const orc_lattice* L, uint32_t* out) {
    if (L->rng != ORC_RNG_MRG32K3A) return -1;
    std::memcpy(out, L->mrg.data(), L->mrg.size() * sizeof(uint32_t));
    return 0;
}

void orc_enable_accept_log(orc_lattice* L, int on) { L->log_accept = on != 0; }
int64_t orc_get_accept_log(const orc_lattice* L, int8_t* out, int64_t nmax) {
    int64_t nn = (int64_t)L->accept_log.size();
    if (out && nmax >= nn) std::memcpy(out, L->accept_log.data(), nn);
    return nn;
}

int orc_update_link(int group, double beta, int nhit, int kind, int reunit, const double* Uc,
                    const double* A, const double* u, double* Uout) {
    int n = group;
    Mat U = from_canonical(n, Uc);
    Mat Am = mat_zero();
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) Am.a[r][c] = cplx(A[2 * (r * n + c)], A[2 * (r * n + c) + 1]);
    ArrayDraws d;
    d.u = u;
    Mat M = mat_mul(n, U, Am);
    Mat R = update_with(n, beta, nhit, kind, U, M, d, nullptr);
    if (reunit) R = reunitarise(n, R);
    to_canonical(n, R, Uout);
    return d.pos;
}

/* ================================================================== */
/* O(N) lambda phi^4 model (the paper's second model family, Sec. 3.3  */
/* and Sec. 5): an N-vector phi(x) per site, N = 1..4.                 */
/* ================================================================== */
/*
 * Action (a reading: the paper names the model and its coupling only; this
 * is the standard hopping-parameter form of the lattice O(N) phi^4 theory,
 * plus a constant source h along component 0 for the external field):
 *   S = sum_x [ -2 kappa sum_{mu} phi(x).phi(x+mu) + phi(x)^2
 *               + lambda (phi(x)^2 - 1)^2 - h phi_0(x) ].
 * Local action of one site with neighbour sum F = sum_mu [phi(x+mu) + phi(x-mu)]:
 *   s(phi) = -2 kappa F.phi + phi.phi + lambda (phi.phi - 1)^2 - h phi_0.
 * Update ("improved" multi-hit Metropolis, Sec. 3.3; NHIT hits per site,
 * Sec. 5): checkerboard, parity 0 sites then parity 1; at each site NHIT
 * successive Metropolis steps with the neighbours fixed: proposal
 * phi' = phi + delta r, r_a = 2 u_a - 1, accepted iff u_acc < exp(-(s(phi') - s(phi))).
 * Draws of hit k of sweep number w at site i:
 *   Philox: counter (i, lattice_id, w, k) -> words w0..w3; u_a from word a
 *           (a < N); u_acc from the 24-bit word formed by the low bytes of
 *           w0, w1, w2 (high to low);
 *   RANLUX: every site update begins a new block; per hit N values for r
 *           then one for u_acc;
 *   MRG32k3a: the site's stream (2^127 apart, as for the SU(N) links),
 *           sequentially: per hit N values for r then one for u_acc;
 *   constant: every uniform = c.
 * Starts: cold phi = (1, 0, ..., 0); hot phi_a = 2 u_a - 1 with Philox counter
 * (i, lattice_id, 0, 0xFFFFFFFF), the first N values of a RANLUX block, or
 * the first N values of the MRG32k3a stream.
 */
struct orc_on {
    int n;
    int d[4];
    int64_t V;
    double kappa, lambda, h, delta;
    int rng;
    double rng_const;
    uint64_t seed;
    int nhit;
    uint32_t lat_id;
    uint64_t sweeps;
    int64_t accepted_last;  // accepted hits of the most recent sweep
    std::vector<double> phi;        // [i][n]
    std::vector<RanluxSite> ranlux;  // one stream per site
    std::vector<uint32_t> mrg;       // 6 words per site
};

static void on_coords(const orc_on* L, int64_t i, int x[4]) {
    for (int m = 0; m < 4; ++m) {
        x[m] = (int)(i % L->d[m]);
        i /= L->d[m];
    }
}
static int64_t on_index(const orc_on* L, const int x[4]) {
    return x[0] + (int64_t)L->d[0] * (x[1] + (int64_t)L->d[1] * (x[2] + (int64_t)L->d[2] * x[3]));
}
static int64_t on_shift(const orc_on* L, int64_t i, int mu, int step) {
    int x[4];
    on_coords(L, i, x);
    x[mu] = (x[mu] + step + L->d[mu]) % L->d[mu];
    return on_index(L, x);
}
static double dot_n(int n, const double* a, const double* b) {
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += a[k] * b[k];
    return s;
}
static double on_local_action(const orc_on* L, const double* F, const double* p) {
    const double p2 = dot_n(L->n, p, p);
    return -2.0 * L->kappa * dot_n(L->n, F, p) + p2 + L->lambda * (p2 - 1.0) * (p2 - 1.0) - L->h * p[0];
}
static double accept_word(uint32_t w0, uint32_t w1, uint32_t w2) {
    return orc_uniform24(((w0 & 0xFFu) << 24) | ((w1 & 0xFFu) << 16) | ((w2 & 0xFFu) << 8));
}

orc_on* orc_on_create(int ncomp, int nx, int ny, int nz, int nt, double kappa, double lambda, double h,
                      double delta, int rng, double rng_const, uint64_t seed, int nhit, uint32_t lattice_id,
                      int start) {
    int dims[4] = {nx, ny, nz, nt};
    if (ncomp < 1 || ncomp > 4) return nullptr;
    for (int m = 0; m < 4; ++m)
        if (dims[m] < 2 || dims[m] % 2) return nullptr;
    if (!std::isfinite(kappa) || !(lambda >= 0.0) || !std::isfinite(lambda) || !std::isfinite(h) ||
        !(delta > 0.0) || !std::isfinite(delta))
        return nullptr;
    if (nhit < 1 || nhit > 1000) return nullptr;
    if (rng < 0 || rng > 3) return nullptr;
    if (rng == ORC_RNG_MRG32K3A && (seed < 1 || seed >= MRG_M2)) return nullptr;
    orc_on* L = new orc_on();
    L->n = ncomp;
    for (int m = 0; m < 4; ++m) L->d[m] = dims[m];
    L->V = (int64_t)nx * ny * nz * nt;
    L->kappa = kappa;
    L->lambda = lambda;
    L->h = h;
    L->delta = delta;
    L->rng = rng;
    L->rng_const = rng_const;
    L->seed = seed;
    L->nhit = nhit;
    L->lat_id = lattice_id;
    L->sweeps = 0;
    L->accepted_last = 0;
    L->phi.assign(L->V * ncomp, 0.0);
    if (rng == ORC_RNG_RANLUX) {
        L->ranlux.resize(L->V);
        for (int64_t i = 0; i < L->V; ++i) L->ranlux[i].eng.seed(ranlux_site_seed(seed, i, lattice_id));
    }
    if (rng == ORC_RNG_MRG32K3A) {
        // site i's stream starts 2^127 i steps into the seed's sequence
        L->mrg.resize(L->V * 6);
        uint32_t st[6];
        orc_mrg_site_state(seed, 0, st);
        M33 j1, j2;
        mrg_pow2(127, j1, j2);
        for (int64_t i = 0; i < L->V; ++i) {
            std::memcpy(&L->mrg[6 * i], st, sizeof(st));
            m33_vec(j1, st, MRG_M1, st);
            m33_vec(j2, st + 3, MRG_M2, st + 3);
        }
    }
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int64_t i = 0; i < L->V; ++i) {
        double* p = &L->phi[i * ncomp];
        if (start == ORC_COLD) {
            p[0] = 1.0;
            continue;
        }
        double u[4];
        if (rng == ORC_RNG_PHILOX) {
            uint32_t c[4] = {(uint32_t)i, lattice_id, 0u, 0xFFFFFFFFu}, o[4];
            orc_philox4x32_10(c, key, o);
            for (int a = 0; a < 4; ++a) u[a] = orc_uniform24(o[a]);
        } else if (rng == ORC_RNG_RANLUX) {
            L->ranlux[i].begin_update();
            for (int a = 0; a < ncomp; ++a) u[a] = L->ranlux[i].next();
        } else if (rng == ORC_RNG_MRG32K3A) {
            for (int a = 0; a < ncomp; ++a) u[a] = orc_uniform24(orc_mrg_next(&L->mrg[6 * i]));
        } else {
            for (int a = 0; a < 4; ++a) u[a] = rng_const;
        }
        for (int a = 0; a < ncomp; ++a) p[a] = 2.0 * u[a] - 1.0;
    }
    return L;
}

void orc_on_destroy(orc_on* L) { delete L; }

/* One sweep: every site of parity 0, then every site of parity 1. */
void orc_on_sweep(orc_on* L, int nsweeps) {
    const int n = L->n;
    const uint32_t key[2] = {(uint32_t)L->seed, (uint32_t)(L->seed >> 32)};
    for (int w = 0; w < nsweeps; ++w) {
        int64_t acc_total = 0;
        for (int p = 0; p < 2; ++p) {
#pragma omp parallel for schedule(static) reduction(+ : acc_total)
            for (int64_t i = 0; i < L->V; ++i) {
                int x[4];
                on_coords(L, i, x);
                if ((x[0] + x[1] + x[2] + x[3]) % 2 != p) continue;
                double F[4] = {0, 0, 0, 0};
                for (int mu = 0; mu < 4; ++mu) {
                    const double* fw = &L->phi[on_shift(L, i, mu, +1) * n];
                    const double* bw = &L->phi[on_shift(L, i, mu, -1) * n];
                    for (int a = 0; a < n; ++a) F[a] += fw[a] + bw[a];
                }
                double* ph = &L->phi[i * n];
                if (L->rng == ORC_RNG_RANLUX) L->ranlux[i].begin_update();
                for (int k = 0; k < L->nhit; ++k) {
                    double u[4], uacc;
                    if (L->rng == ORC_RNG_PHILOX) {
                        uint32_t c[4] = {(uint32_t)i, L->lat_id, (uint32_t)L->sweeps, (uint32_t)k}, o[4];
                        orc_philox4x32_10(c, key, o);
                        for (int a = 0; a < 4; ++a) u[a] = orc_uniform24(o[a]);
                        uacc = accept_word(o[0], o[1], o[2]);
                    } else if (L->rng == ORC_RNG_RANLUX) {
                        for (int a = 0; a < n; ++a) u[a] = L->ranlux[i].next();
                        uacc = L->ranlux[i].next();
                    } else if (L->rng == ORC_RNG_MRG32K3A) {
                        for (int a = 0; a < n; ++a) u[a] = orc_uniform24(orc_mrg_next(&L->mrg[6 * i]));
                        uacc = orc_uniform24(orc_mrg_next(&L->mrg[6 * i]));
                    } else {
                        for (int a = 0; a < 4; ++a) u[a] = L->rng_const;
                        uacc = L->rng_const;
                    }
                    double trial[4];
                    for (int a = 0; a < n; ++a) trial[a] = ph[a] + L->delta * (2.0 * u[a] - 1.0);
                    const double dS = on_local_action(L, F, trial) - on_local_action(L, F, ph);
                    if (uacc < std::exp(-dS)) {
                        for (int a = 0; a < n; ++a) ph[a] = trial[a];
                        ++acc_total;
                    }
                }
            }
        }
        L->accepted_last = acc_total;
        L->sweeps += 1;
    }
}

/* out = { <phi^2>, <phi(x).phi(x+mu)> over sites and the 4 directions,
 *         <(phi^2 - 1)^2>, <phi_0>, <phi_1>, <phi_2>, <phi_3> } (components
 * beyond N are 0).  Compensated sums in site order. */
void orc_on_measure(const orc_on* L, double out[7]) {
    const int n = L->n;
    std::vector<double> p2(L->V), lk(L->V), q(L->V), m[4];
    for (int a = 0; a < 4; ++a) m[a].assign(L->V, 0.0);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < L->V; ++i) {
        const double* ph = &L->phi[i * n];
        const double s2 = dot_n(n, ph, ph);
        p2[i] = s2;
        q[i] = (s2 - 1.0) * (s2 - 1.0);
        double l = 0.0;
        for (int mu = 0; mu < 4; ++mu) l += dot_n(n, ph, &L->phi[on_shift(L, i, mu, +1) * n]);
        lk[i] = l;
        for (int a = 0; a < n; ++a) m[a][i] = ph[a];
    }
    const double V = (double)L->V;
    out[0] = neumaier(p2) / V;
    out[1] = neumaier(lk) / (4.0 * V);
    out[2] = neumaier(q) / V;
    for (int a = 0; a < 4; ++a) out[3 + a] = neumaier(m[a]) / V;
}

void orc_on_get_field(const orc_on* L, double* out) { std::memcpy(out, L->phi.data(), L->phi.size() * sizeof(double)); }
void orc_on_set_field(orc_on* L, const double* in) { std::memcpy(L->phi.data(), in, L->phi.size() * sizeof(double)); }
uint64_t orc_on_sweeps(const orc_on* L) { return L->sweeps; }
int orc_on_get_mrg_states(const orc_on* L, uint32_t* out) {
    if (L->rng != ORC_RNG_MRG32K3A) return -1;
    std::memcpy(out, L->mrg.data(), L->mrg.size() * sizeof(uint32_t));
    return 0;
}
double orc_on_acceptance(const orc_on* L) {
    return (double)L->accepted_last / ((double)L->V * (double)L->nhit);
}
