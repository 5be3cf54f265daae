// Device-side building blocks for gfx950: complex SU(3) and quaternion SU(2)
// algebra, the per-site random streams and the parity-split link layout.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lat_types.hpp"

#define LAT_DEV __device__ __forceinline__

namespace latdev {

constexpr double TWO_PI = 6.283185307179586476925286766559;

// ---------------------------------------------------------------------------
// complex numbers and 3x3 matrices (row-major)
// ---------------------------------------------------------------------------
template <class T>
struct cx {
    T re, im;
};
template <class T>
LAT_DEV cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <class T>
LAT_DEV cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <class T>
LAT_DEV cx<T> cmul(cx<T> a, cx<T> b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
// conj(a) * b
template <class T>
LAT_DEV cx<T> cjmul(cx<T> a, cx<T> b) { return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re}; }
// a * conj(b)
template <class T>
LAT_DEV cx<T> cmulj(cx<T> a, cx<T> b) { return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im}; }
template <class T>
LAT_DEV cx<T> conj(cx<T> a) { return {a.re, -a.im}; }

template <class T>
struct m3 {
    cx<T> e[3][3];
};

template <class T>
LAT_DEV m3<T> zero3() {
    m3<T> r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) r.e[i][j] = {T(0), T(0)};
    return r;
}

// Complex multiply-accumulate written as four fused multiply-adds per term
// (without it the compiler keeps a separate multiply and add per product,
// half again as many VALU instructions).
LAT_DEV float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
LAT_DEV double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }
// s += a * b
template <class T>
LAT_DEV void cmac(cx<T>& s, cx<T> a, cx<T> b) {
    s.re = fmad(a.re, b.re, s.re);
    s.re = fmad(-a.im, b.im, s.re);
    s.im = fmad(a.re, b.im, s.im);
    s.im = fmad(a.im, b.re, s.im);
}
// s += a * conj(b)
template <class T>
LAT_DEV void cmacj(cx<T>& s, cx<T> a, cx<T> b) {
    s.re = fmad(a.re, b.re, s.re);
    s.re = fmad(a.im, b.im, s.re);
    s.im = fmad(a.im, b.re, s.im);
    s.im = fmad(-a.re, b.im, s.im);
}
// s += conj(a) * b
template <class T>
LAT_DEV void cjmac(cx<T>& s, cx<T> a, cx<T> b) {
    s.re = fmad(a.re, b.re, s.re);
    s.re = fmad(a.im, b.im, s.re);
    s.im = fmad(a.re, b.im, s.im);
    s.im = fmad(-a.im, b.re, s.im);
}
// first term of a sum: a * b
template <class T>
LAT_DEV cx<T> cmul0(cx<T> a, cx<T> b) { return {fmad(-a.im, b.im, a.re * b.re), fmad(a.im, b.re, a.re * b.im)}; }
template <class T>
LAT_DEV cx<T> cmulj0(cx<T> a, cx<T> b) { return {fmad(a.im, b.im, a.re * b.re), fmad(-a.re, b.im, a.im * b.re)}; }
template <class T>
LAT_DEV cx<T> cjmul0(cx<T> a, cx<T> b) { return {fmad(a.im, b.im, a.re * b.re), fmad(-a.im, b.re, a.re * b.im)}; }

// A * B
template <class T>
LAT_DEV m3<T> mul_nn(const m3<T>& a, const m3<T>& b) {
    m3<T> r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<T> s = cmul0(a.e[i][0], b.e[0][j]);
            cmac(s, a.e[i][1], b.e[1][j]);
            cmac(s, a.e[i][2], b.e[2][j]);
            r.e[i][j] = s;
        }
    return r;
}
// A * B^dagger
template <class T>
LAT_DEV m3<T> mul_na(const m3<T>& a, const m3<T>& b) {
    m3<T> r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<T> s = cmulj0(a.e[i][0], b.e[j][0]);
            cmacj(s, a.e[i][1], b.e[j][1]);
            cmacj(s, a.e[i][2], b.e[j][2]);
            r.e[i][j] = s;
        }
    return r;
}
// A^dagger * B
template <class T>
LAT_DEV m3<T> mul_an(const m3<T>& a, const m3<T>& b) {
    m3<T> r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<T> s = cjmul0(a.e[0][i], b.e[0][j]);
            cjmac(s, a.e[1][i], b.e[1][j]);
            cjmac(s, a.e[2][i], b.e[2][j]);
            r.e[i][j] = s;
        }
    return r;
}
// Rows 0 and 1 of A * B^dagger and of A * B (row 2 is left as it is: for a
// product of SU(3) matrices it is conj(row 0 x row 1), see third_row).
template <class T>
LAT_DEV void mul_na_rows01(m3<T>& r, const m3<T>& a, const m3<T>& b) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<T> s = cmulj0(a.e[i][0], b.e[j][0]);
            cmacj(s, a.e[i][1], b.e[j][1]);
            cmacj(s, a.e[i][2], b.e[j][2]);
            r.e[i][j] = s;
        }
}
template <class T>
LAT_DEV void mul_nn_rows01(m3<T>& r, const m3<T>& a, const m3<T>& b) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<T> s = cmul0(a.e[i][0], b.e[0][j]);
            cmac(s, a.e[i][1], b.e[1][j]);
            cmac(s, a.e[i][2], b.e[2][j]);
            r.e[i][j] = s;
        }
}
// C += A * B^dagger
template <class T>
LAT_DEV void mac_na(m3<T>& c, const m3<T>& a, const m3<T>& b) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int k = 0; k < 3; ++k) cmacj(c.e[i][j], a.e[i][k], b.e[j][k]);
}
// C += A^dagger * B
template <class T>
LAT_DEV void mac_an(m3<T>& c, const m3<T>& a, const m3<T>& b) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int k = 0; k < 3; ++k) cjmac(c.e[i][j], a.e[k][i], b.e[k][j]);
}
template <class T>
LAT_DEV void acc3(m3<T>& a, const m3<T>& b) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) a.e[i][j] = a.e[i][j] + b.e[i][j];
}
template <class T>
LAT_DEV T re_tr(const m3<T>& a) { return a.e[0][0].re + a.e[1][1].re + a.e[2][2].re; }
// Re Tr(A * B^dagger) without forming the product
template <class T>
LAT_DEV T re_tr_na(const m3<T>& a, const m3<T>& b) {
    T s = T(0);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) s += a.e[i][k].re * b.e[i][k].re + a.e[i][k].im * b.e[i][k].im;
    return s;
}
template <class T>
LAT_DEV m3<T> identity3() {
    m3<T> r = zero3<T>();
    r.e[0][0].re = r.e[1][1].re = r.e[2][2].re = T(1);
    return r;
}
template <class To, class From>
LAT_DEV m3<To> cast3(const m3<From>& a) {
    m3<To> r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) r.e[i][j] = {To(a.e[i][j].re), To(a.e[i][j].im)};
    return r;
}
// row 3 = conj(row1 x row2): completes two orthonormal rows to det = 1
template <class T>
LAT_DEV cx<T> conj_cross(cx<T> a, cx<T> b, cx<T> c, cx<T> d) {  // conj(a b - c d)
    cx<T> t = cmul0(a, b);
    t.re = fmad(-c.re, d.re, t.re);
    t.re = fmad(c.im, d.im, t.re);
    t.im = fmad(-c.re, d.im, t.im);
    t.im = fmad(-c.im, d.re, t.im);
    return {t.re, -t.im};
}
template <class T>
LAT_DEV void third_row(m3<T>& a) {
    a.e[2][0] = conj_cross(a.e[0][1], a.e[1][2], a.e[0][2], a.e[1][1]);
    a.e[2][1] = conj_cross(a.e[0][2], a.e[1][0], a.e[0][0], a.e[1][2]);
    a.e[2][2] = conj_cross(a.e[0][0], a.e[1][1], a.e[0][1], a.e[1][0]);
}
// Gram-Schmidt on rows 1-2, then row 3 from the cross product (FP64)
LAT_DEV void reunit3(m3<double>& a) {
    double n1 = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) n1 += a.e[0][c].re * a.e[0][c].re + a.e[0][c].im * a.e[0][c].im;
    n1 = 1.0 / sqrt(n1);
#pragma unroll
    for (int c = 0; c < 3; ++c) a.e[0][c] = {a.e[0][c].re * n1, a.e[0][c].im * n1};
    cx<double> d = {0.0, 0.0};
#pragma unroll
    for (int c = 0; c < 3; ++c) d = d + cjmul(a.e[0][c], a.e[1][c]);
#pragma unroll
    for (int c = 0; c < 3; ++c) a.e[1][c] = a.e[1][c] - cmul(d, a.e[0][c]);
    double n2 = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) n2 += a.e[1][c].re * a.e[1][c].re + a.e[1][c].im * a.e[1][c].im;
    n2 = 1.0 / sqrt(n2);
#pragma unroll
    for (int c = 0; c < 3; ++c) a.e[1][c] = {a.e[1][c].re * n2, a.e[1][c].im * n2};
    third_row(a);
}

// ---------------------------------------------------------------------------
// quaternions q0 + i(q1 s1 + q2 s2 + q3 s3) for SU(2)
// ---------------------------------------------------------------------------
template <class T>
struct qt {
    T q0, q1, q2, q3;
};
// a * b
template <class T>
LAT_DEV qt<T> qmul(qt<T> a, qt<T> b) {
    return {a.q0 * b.q0 - a.q1 * b.q1 - a.q2 * b.q2 - a.q3 * b.q3,
            a.q0 * b.q1 + b.q0 * a.q1 - (a.q2 * b.q3 - a.q3 * b.q2),
            a.q0 * b.q2 + b.q0 * a.q2 - (a.q3 * b.q1 - a.q1 * b.q3),
            a.q0 * b.q3 + b.q0 * a.q3 - (a.q1 * b.q2 - a.q2 * b.q1)};
}
template <class T>
LAT_DEV qt<T> qdag(qt<T> a) { return {a.q0, -a.q1, -a.q2, -a.q3}; }
// a * b^dagger
template <class T>
LAT_DEV qt<T> qmul_na(qt<T> a, qt<T> b) { return qmul(a, qdag(b)); }
template <class T>
LAT_DEV qt<T> qadd(qt<T> a, qt<T> b) { return {a.q0 + b.q0, a.q1 + b.q1, a.q2 + b.q2, a.q3 + b.q3}; }
template <class T>
LAT_DEV T qnorm2(qt<T> a) { return a.q0 * a.q0 + a.q1 * a.q1 + a.q2 * a.q2 + a.q3 * a.q3; }

// Left multiplication of rows a, b of a 3x3 matrix by the SU(2) element r
// embedded in the (a,b) block: (r00 r01; r10 r11) =
// (r0 + i r3, r2 + i r1; -r2 + i r1, r0 - i r3).
template <class T>
LAT_DEV void left_mul_block(m3<T>& m, int a, int b, qt<T> r) {
    const cx<T> r00 = {r.q0, r.q3}, r01 = {r.q2, r.q1}, r10 = {-r.q2, r.q1}, r11 = {r.q0, -r.q3};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        cx<T> x = m.e[a][c], y = m.e[b][c];
        m.e[a][c] = cmul(r00, x) + cmul(r01, y);
        m.e[b][c] = cmul(r10, x) + cmul(r11, y);
    }
}
// Quaternion (SU(2) projection) of the (a,b) block of a 3x3 matrix.
template <class T>
LAT_DEV qt<T> block_quat(const m3<T>& m, int a, int b) {
    return {T(0.5) * (m.e[a][a].re + m.e[b][b].re), T(0.5) * (m.e[a][b].im + m.e[b][a].im),
            T(0.5) * (m.e[a][b].re - m.e[b][a].re), T(0.5) * (m.e[a][a].im - m.e[b][b].im)};
}

// ---------------------------------------------------------------------------
// random streams
// ---------------------------------------------------------------------------
// 24 high bits, centred: exact in FP32 and FP64, never 0 or 1
LAT_DEV double u24(uint32_t w) { return ((double)(w >> 8) + 0.5) * (1.0 / 16777216.0); }

struct u4 {
    uint32_t x, y, z, w;
};
// Philox4x32-10 (Salmon et al., SC'11)
LAT_DEV u4 philox10(u4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32->64 multiply per word gives both halves (a single
        // v_mad_u64_u32 instead of separate low and high multiplies)
        const uint64_t m0 = (uint64_t)0xD2511F53u * c.x, m1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t lo0 = (uint32_t)m0, hi0 = (uint32_t)(m0 >> 32);
        const uint32_t lo1 = (uint32_t)m1, hi1 = (uint32_t)(m1 >> 32);
        c = {hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// MRG32k3a step on a register-resident state; returns z in [1, m1].
struct mrg_state {
    uint32_t s[6];
};
LAT_DEV uint32_t mrg_step(mrg_state& st) {
    const uint64_t m1 = 4294967087ull, m2 = 4294944443ull;
    // -a * x mod m == a * (m - x) mod m keeps every term non-negative (< 2^54)
    uint64_t p1 = (1403580ull * st.s[1] + 810728ull * (m1 - st.s[0])) % m1;
    uint64_t p2 = (527612ull * st.s[5] + 1370589ull * (m2 - st.s[3])) % m2;
    st.s[0] = st.s[1];
    st.s[1] = st.s[2];
    st.s[2] = (uint32_t)p1;
    st.s[3] = st.s[4];
    st.s[4] = st.s[5];
    st.s[5] = (uint32_t)p2;
    return (uint32_t)(p1 > p2 ? p1 - p2 : p1 + m1 - p2);
}

// Uniforms of one link update.  Philox addresses slots by
// (site, lattice, 4*h + mu, g*(NHIT+1) + t); MRG draws sequentially.
template <int RNG>
struct draws;

template <>
struct draws<LAT_RNG_PHILOX_I> {
    uint32_t site, lat, word2, k0, k1;
    int nhit;
    LAT_DEV void try4(int g, int t, double R[4]) {
        u4 o = philox10({site, lat, word2, (uint32_t)(g * (nhit + 1) + t)}, k0, k1);
        R[0] = u24(o.x);
        R[1] = u24(o.y);
        R[2] = u24(o.z);
        R[3] = u24(o.w);
    }
    LAT_DEV void dir2(int g, double D[2]) {
        u4 o = philox10({site, lat, word2, (uint32_t)(g * (nhit + 1) + nhit)}, k0, k1);
        D[0] = u24(o.x);
        D[1] = u24(o.y);
    }
};
template <>
struct draws<LAT_RNG_MRG_I> {
    mrg_state st;
    LAT_DEV void try4(int, int, double R[4]) {
#pragma unroll
        for (int k = 0; k < 4; ++k) R[k] = u24(mrg_step(st));
    }
    LAT_DEV void dir2(int, double D[2]) {
        D[0] = u24(mrg_step(st));
        D[1] = u24(mrg_step(st));
    }
};
// RANLUX, luxury level 3: subtract-with-borrow x_n = x_{n-10} - x_{n-24} - c
// mod 2^24; of every 223 outputs the first 24 are used.  b[24] holds the
// last 24 outputs oldest first, so one in-place round of 24 steps reads
// x_{n-10} at b[(k+14) % 24] (an old value for k < 10, a new one after) and
// x_{n-24} at b[k], and leaves b oldest first again.
// One step: with 24-bit operands in 32-bit registers the borrow out of the
// 32-bit subtraction a - b - c is exactly the generator's carry (a < b + c),
// so a subtract-with-borrow instruction yields both, and a mask the value.
LAT_DEV uint32_t swb_step(uint32_t a, uint32_t b, uint32_t& c) {
    unsigned int borrow;
    const uint32_t y = __builtin_subc(a, b, c, &borrow);
    c = borrow;
    return y & 0xFFFFFFu;
}
LAT_DEV void swb_round(uint32_t (&b)[24], uint32_t& c) {
#pragma unroll
    for (int k = 0; k < 24; ++k) b[k] = swb_step(b[(k + 14) % 24], b[k], c);
}
// From the last delivered block to the next one: skip the other 199 outputs
// of the current group of 223 (8 rounds and 7 steps, after which b is
// rotated back to oldest first), then one round gives the 24 next outputs.
// The first block after seeding follows the seed words directly.
LAT_DEV void ranlux_next_block(uint32_t (&b)[24], uint32_t& c, bool skip) {
    if (skip) {
        for (int r = 0; r < 8; ++r) swb_round(b, c);
#pragma unroll
        for (int k = 0; k < 7; ++k) b[k] = swb_step(b[k + 14], b[k], c);
        uint32_t t[24];
#pragma unroll
        for (int j = 0; j < 24; ++j) t[j] = b[(j + 7) % 24];
#pragma unroll
        for (int j = 0; j < 24; ++j) b[j] = t[j];
    }
    swb_round(b, c);
}
// The current block lives in LDS (word j of this thread at lds[j * stride])
// because draws index it with a per-lane position; a link update that
// needs more than 24 values moves on to the next block.
template <>
struct draws<LAT_RNG_RANLUX_I> {
    uint32_t* lds;
    int stride;
    uint32_t c;
    int idx;
    LAT_DEV uint32_t next() {
        if (idx == 24) {
            uint32_t b[24];
#pragma unroll
            for (int j = 0; j < 24; ++j) b[j] = lds[j * stride];
            ranlux_next_block(b, c, true);
#pragma unroll
            for (int j = 0; j < 24; ++j) lds[j * stride] = b[j];
            idx = 0;
        }
        return lds[(idx++) * stride];
    }
    LAT_DEV void try4(int, int, double R[4]) {
#pragma unroll
        for (int k = 0; k < 4; ++k) R[k] = u24(next() << 8);
    }
    LAT_DEV void dir2(int, double D[2]) {
        D[0] = u24(next() << 8);
        D[1] = u24(next() << 8);
    }
};
template <>
struct draws<LAT_RNG_CONST_I> {
    double c;
    LAT_DEV void try4(int, int, double R[4]) { R[0] = R[1] = R[2] = R[3] = c; }
    LAT_DEV void dir2(int, double D[2]) { D[0] = D[1] = c; }
};

// Kennedy-Pendleton: x0 with density sqrt(1-x0^2) exp(alpha x0).
// Returns the accepted try or -1 (then x = 1).
template <class DR>
LAT_DEV int kp(double alpha, int nhit, DR& d, int g, qt<double>& x) {
    for (int t = 0; t < nhit; ++t) {
        double R[4];
        d.try4(g, t, R);
        const double c = cospi(2.0 * R[1]);  // cos(2 pi R2), exact argument
        const double lam2 = -(log(R[0]) + c * c * log(R[2])) / (2.0 * alpha);
        if (R[3] * R[3] <= 1.0 - lam2) {
            double D[2];
            d.dir2(g, D);
            const double s = 2.0 * sqrt(lam2 * (1.0 - lam2));
            const double ct = 2.0 * D[0] - 1.0;
            const double st = sqrt(1.0 - ct * ct);
            double sp, cp;
            sincospi(2.0 * D[1], &sp, &cp);  // phi = 2 pi R6
            x = {1.0 - 2.0 * lam2, s * st * cp, s * st * sp, s * ct};
            return t;
        }
    }
    x = {1.0, 0.0, 0.0, 0.0};
    return -1;
}

// First try of a KP draw and the direction of the SU(2) element, prepared
// from the random numbers alone (they do not depend on the links): the
// transcendental work then overlaps the staple's memory traffic.  Only for
// counter-addressed or constant generators, whose draws do not depend on how
// many tries earlier subgroups took.
struct kp_first {
    double num;             // ln R1 + cos^2(2 pi R2) ln R3 of try 0
    double r4sq;            // R4^2 of try 0
    double dx, dy, dz;      // unit direction of (a1, a2, a3)
};
template <class DR>
LAT_DEV kp_first kp_prepare(DR& d, int g) {
    kp_first f;
    double R[4], D[2];
    d.try4(g, 0, R);
    const double c = cospi(2.0 * R[1]);  // cos(2 pi R2), exact argument
    f.num = log(R[0]) + c * c * log(R[2]);
    f.r4sq = R[3] * R[3];
    d.dir2(g, D);
    const double ct = 2.0 * D[0] - 1.0;
    const double st = sqrt(1.0 - ct * ct);
    double sp, cp;
    sincospi(2.0 * D[1], &sp, &cp);  // phi = 2 pi R6
    f.dx = st * cp;
    f.dy = st * sp;
    f.dz = ct;
    return f;
}
// The same draw as kp(), starting from a prepared first try.
template <class DR>
LAT_DEV int kp_prepared(double alpha, int nhit, DR& d, int g, const kp_first& f, qt<double>& x) {
    double lam2 = -f.num / (2.0 * alpha);
    int t = 0;
    if (!(f.r4sq <= 1.0 - lam2)) {
        for (t = 1; t < nhit; ++t) {
            double R[4];
            d.try4(g, t, R);
            const double c = cospi(2.0 * R[1]);  // cos(2 pi R2), exact argument
            lam2 = -(log(R[0]) + c * c * log(R[2])) / (2.0 * alpha);
            if (R[3] * R[3] <= 1.0 - lam2) break;
        }
        if (t == nhit) {
            x = {1.0, 0.0, 0.0, 0.0};
            return -1;
        }
    }
    const double s = 2.0 * sqrt(lam2 * (1.0 - lam2));
    x = {1.0 - 2.0 * lam2, s * f.dx, s * f.dy, s * f.dz};
    return t;
}

// ---------------------------------------------------------------------------
// geometry of the parity-split layout
// ---------------------------------------------------------------------------
struct coord4 {
    int x, y, z, t;
};
// half-lattice index s of parity p -> coordinates
LAT_DEV coord4 decode(const LatGeom& g, int64_t s, int p) {
    int64_t r = s / g.nxh;
    const int xh = (int)(s - r * g.nxh);
    const int64_t r2 = r / g.ny;
    const int y = (int)(r - r2 * g.ny);
    const int t = (int)(r2 / g.nz);
    const int z = (int)(r2 - (int64_t)t * g.nz);
    const int x = 2 * xh + ((p + y + z + t) & 1);
    return {x, y, z, t};
}
LAT_DEV int64_t half_index(const LatGeom& g, coord4 c) {
    return (int64_t)(c.x >> 1) + (int64_t)g.nxh * (c.y + (int64_t)g.ny * (c.z + (int64_t)g.nz * c.t));
}
LAT_DEV int64_t canon_index(const LatGeom& g, coord4 c) {
    return c.x + (int64_t)g.nx * (c.y + (int64_t)g.ny * (c.z + (int64_t)g.nz * c.t));
}
LAT_DEV coord4 step(const LatGeom& g, coord4 c, int mu, int d) {
    switch (mu) {
        case 0: c.x += d; c.x = c.x < 0 ? c.x + g.nx : (c.x >= g.nx ? c.x - g.nx : c.x); break;
        case 1: c.y += d; c.y = c.y < 0 ? c.y + g.ny : (c.y >= g.ny ? c.y - g.ny : c.y); break;
        case 2: c.z += d; c.z = c.z < 0 ? c.z + g.nz : (c.z >= g.nz ? c.z - g.nz : c.z); break;
        default: c.t += d; c.t = c.t < 0 ? c.t + g.nt : (c.t >= g.nt ? c.t - g.nt : c.t); break;
    }
    return c;
}

// 32-bit site arithmetic for the sweep kernels.  A half lattice has fewer
// than 2^31 sites on any device (the host refuses larger lattices), so half
// indices and coordinates fit 32 bits; neighbour indices follow from the
// site's own index by a stride and a wrap-around correction instead of a
// full re-encoding.
struct site32 {
    int x, y, z, t;  // coordinates
    uint32_t s;      // half-lattice index
};
LAT_DEV site32 site_of(const LatGeom& g, uint32_t s, int p) {
    const uint32_t nxh = (uint32_t)g.nxh, ny = (uint32_t)g.ny, nz = (uint32_t)g.nz;
    const uint32_t r = s / nxh;
    const uint32_t xh = s - r * nxh;
    const uint32_t r2 = r / ny;
    const uint32_t y = r - r2 * ny;
    const uint32_t t = r2 / nz;
    const uint32_t z = r2 - t * nz;
    site32 c;
    c.y = (int)y;
    c.z = (int)z;
    c.t = (int)t;
    c.x = 2 * (int)xh + (int)((p + y + z + t) & 1);
    c.s = s;
    return c;
}
// The neighbour c + d mu-hat (d = +-1), coordinates and half index.
LAT_DEV site32 site_step(const LatGeom& g, site32 c, int mu, int d) {
    switch (mu) {
        case 0: {
            int x = c.x + d;
            x = x < 0 ? x + g.nx : (x >= g.nx ? x - g.nx : x);
            c.s = c.s - (uint32_t)(c.x >> 1) + (uint32_t)(x >> 1);
            c.x = x;
            break;
        }
        case 1: {
            const uint32_t st = (uint32_t)g.nxh;
            int y = c.y + d;
            if (y < 0) {
                y += g.ny;
                c.s += (uint32_t)(g.ny - 1) * st;
            } else if (y >= g.ny) {
                y -= g.ny;
                c.s -= (uint32_t)(g.ny - 1) * st;
            } else {
                c.s = d > 0 ? c.s + st : c.s - st;
            }
            c.y = y;
            break;
        }
        case 2: {
            const uint32_t st = (uint32_t)g.nxh * (uint32_t)g.ny;
            int z = c.z + d;
            if (z < 0) {
                z += g.nz;
                c.s += (uint32_t)(g.nz - 1) * st;
            } else if (z >= g.nz) {
                z -= g.nz;
                c.s -= (uint32_t)(g.nz - 1) * st;
            } else {
                c.s = d > 0 ? c.s + st : c.s - st;
            }
            c.z = z;
            break;
        }
        default: {
            const uint32_t st = (uint32_t)g.nxh * (uint32_t)g.ny * (uint32_t)g.nz;
            int t = c.t + d;
            if (t < 0) {
                t += g.nt;
                c.s += (uint32_t)(g.nt - 1) * st;
            } else if (t >= g.nt) {
                t -= g.nt;
                c.s -= (uint32_t)(g.nt - 1) * st;
            } else {
                c.s = d > 0 ? c.s + st : c.s - st;
            }
            c.t = t;
            break;
        }
    }
    return c;
}
LAT_DEV coord4 coords(const site32& c) { return {c.x, c.y, c.z, c.t}; }

// Background phase theta of link (c, mu): B = exp(i theta T).
LAT_DEV double bg_theta(const LatGeom& g, int flux, coord4 c, int mu) {
    if (flux == 0 || mu > 1) return 0.0;
    const double phi = TWO_PI * (double)flux / (double)(g.nx * g.ny);
    if (mu == 1) return phi * (double)c.x;
    if (c.x == g.nx - 1) return -phi * (double)(g.nx * c.y);
    return 0.0;
}

// ---------------------------------------------------------------------------
// storage forms: each (parity, mu) holds NP planes of 8- or 16-byte vectors,
// every plane a contiguous array over the padded half lattice.
// ---------------------------------------------------------------------------
// Element k of a link: plane k starts plane_bytes * k after the first plane;
// the per-thread part of the address is a 32-bit byte offset (so the
// uniform plane base stays in scalar registers).
template <class V>
LAT_DEV V ld_plane(const char* base, int64_t plane_bytes, int k, uint32_t off) {
    return *reinterpret_cast<const V*>(base + k * plane_bytes + off);
}
template <class V>
LAT_DEV void st_plane(char* base, int64_t plane_bytes, int k, uint32_t off, V v) {
    *reinterpret_cast<V*>(base + k * plane_bytes + off) = v;
}

struct st_f64 {  // SU(3), 18 doubles: 9 planes of (re, im)
    using vec = double2;  // one plane element
    using real = double;
    using mat = m3<double>;
    static constexpr int NP = 9;
    static constexpr int VB = 16;
    static constexpr bool TWO_ROWS = false;  // all three rows are stored
    // rows 0 and 1 only (row 2 zero): the first factor of a two-row product
    LAT_DEV static mat load_rows01(const char* base, int64_t plane_stride, int64_t s) {
        const uint32_t off = (uint32_t)s * VB;
        const int64_t pb = plane_stride * VB;
        mat m;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const double2 v = ld_plane<double2>(base, pb, k, off);
            m.e[k / 3][k % 3] = {v.x, v.y};
        }
        m.e[2][0] = m.e[2][1] = m.e[2][2] = {double(0), double(0)};
        return m;
    }
    LAT_DEV static mat load(const char* base, int64_t plane_stride, int64_t s) {
        const uint32_t off = (uint32_t)s * VB;
        const int64_t pb = plane_stride * VB;
        mat m;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const double2 v = ld_plane<double2>(base, pb, k, off);
            m.e[k / 3][k % 3] = {v.x, v.y};
        }
        return m;
    }
    LAT_DEV static void store(char* base, int64_t plane_stride, int64_t s, const mat& m) {
        const uint32_t off = (uint32_t)s * VB;
        const int64_t pb = plane_stride * VB;
#pragma unroll
        for (int k = 0; k < 9; ++k) st_plane(base, pb, k, off, make_double2(m.e[k / 3][k % 3].re, m.e[k / 3][k % 3].im));
    }
};
struct st_f32 {  // SU(3), 18 floats: 9 planes of (re, im)
    using vec = float2;  // one plane element
    using real = float;
    using mat = m3<float>;
    static constexpr int NP = 9;
    static constexpr int VB = 8;
    static constexpr bool TWO_ROWS = false;
    // rows 0 and 1 only (row 2 zero): the first factor of a two-row product
    LAT_DEV static mat load_rows01(const char* base, int64_t plane_stride, int64_t s) {
        const uint32_t off = (uint32_t)s * VB;
        const int64_t pb = plane_stride * VB;
        mat m;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const float2 v = ld_plane<float2>(base, pb, k, off);
            m.e[k / 3][k % 3] = {v.x, v.y};
        }
        m.e[2][0] = m.e[2][1] = m.e[2][2] = {float(0), float(0)};
        return m;
    }
    LAT_DEV static mat load(const char* base, int64_t plane_stride, int64_t s) {
        const uint32_t off = (uint32_t)s * VB;
        const int64_t pb = plane_stride * VB;
        mat m;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const float2 v = ld_plane<float2>(base, pb, k, off);
            m.e[k / 3][k % 3] = {v.x, v.y};
        }
        return m;
    }
    LAT_DEV static void store(char* base, int64_t plane_stride, int64_t s, const mat& m) {
        const uint32_t off = (uint32_t)s * VB;
        const int64_t pb = plane_stride * VB;
#pragma unroll
        for (int k = 0; k < 9; ++k) st_plane(base, pb, k, off, make_float2(m.e[k / 3][k % 3].re, m.e[k / 3][k % 3].im));
    }
};
struct st_f32c12 {  // SU(3), rows 1-2 as 3 planes of float4; row 3 rebuilt
    using vec = float4;  // one plane element
    using real = float;
    using mat = m3<float>;
    static constexpr int NP = 3;
    static constexpr int VB = 16;
    static constexpr bool TWO_ROWS = true;  // only rows 0 and 1 are stored
    // rows 0 and 1 only (row 2 zero)
    LAT_DEV static mat load_rows01(const char* base, int64_t plane_stride, int64_t s) {
        const uint32_t off = (uint32_t)s * VB;
        const int64_t pb = plane_stride * VB;
        const float4 a = ld_plane<float4>(base, pb, 0, off);
        const float4 b = ld_plane<float4>(base, pb, 1, off);
        const float4 c = ld_plane<float4>(base, pb, 2, off);
        mat m;
        m.e[0][0] = {a.x, a.y};
        m.e[0][1] = {a.z, a.w};
        m.e[0][2] = {b.x, b.y};
        m.e[1][0] = {b.z, b.w};
        m.e[1][1] = {c.x, c.y};
        m.e[1][2] = {c.z, c.w};
        m.e[2][0] = m.e[2][1] = m.e[2][2] = {0.f, 0.f};
        return m;
    }
    LAT_DEV static mat load(const char* base, int64_t plane_stride, int64_t s) {
        mat m = load_rows01(base, plane_stride, s);
        third_row(m);
        return m;
    }
    LAT_DEV static void store(char* base, int64_t plane_stride, int64_t s, const mat& m) {
        const uint32_t off = (uint32_t)s * VB;
        const int64_t pb = plane_stride * VB;
        st_plane(base, pb, 0, off, make_float4(m.e[0][0].re, m.e[0][0].im, m.e[0][1].re, m.e[0][1].im));
        st_plane(base, pb, 1, off, make_float4(m.e[0][2].re, m.e[0][2].im, m.e[1][0].re, m.e[1][0].im));
        st_plane(base, pb, 2, off, make_float4(m.e[1][1].re, m.e[1][1].im, m.e[1][2].re, m.e[1][2].im));
    }
};
struct st_f64c12 {  // SU(3), rows 1-2 as 6 planes of (re, im) doubles; row 3 rebuilt
    using vec = double2;  // one plane element
    using real = double;
    using mat = m3<double>;
    static constexpr int NP = 6;
    static constexpr int VB = 16;
    static constexpr bool TWO_ROWS = true;  // only rows 0 and 1 are stored
    // rows 0 and 1 only (row 2 zero)
    LAT_DEV static mat load_rows01(const char* base, int64_t plane_stride, int64_t s) {
        const uint32_t off = (uint32_t)s * VB;
        const int64_t pb = plane_stride * VB;
        mat m;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const double2 v = ld_plane<double2>(base, pb, k, off);
            m.e[k / 3][k % 3] = {v.x, v.y};
        }
        m.e[2][0] = m.e[2][1] = m.e[2][2] = {0.0, 0.0};
        return m;
    }
    LAT_DEV static mat load(const char* base, int64_t plane_stride, int64_t s) {
        mat m = load_rows01(base, plane_stride, s);
        third_row(m);
        return m;
    }
    LAT_DEV static void store(char* base, int64_t plane_stride, int64_t s, const mat& m) {
        const uint32_t off = (uint32_t)s * VB;
        const int64_t pb = plane_stride * VB;
#pragma unroll
        for (int k = 0; k < 6; ++k) st_plane(base, pb, k, off, make_double2(m.e[k / 3][k % 3].re, m.e[k / 3][k % 3].im));
    }
};
struct sq_f64 {  // SU(2), 4 doubles: 2 planes of double2
    using vec = double2;  // one plane element
    using real = double;
    using mat = qt<double>;
    static constexpr int NP = 2;
    static constexpr int VB = 16;
    LAT_DEV static mat load(const char* base, int64_t plane_stride, int64_t s) {
        const uint32_t off = (uint32_t)s * VB;
        const int64_t pb = plane_stride * VB;
        const double2 a = ld_plane<double2>(base, pb, 0, off), b = ld_plane<double2>(base, pb, 1, off);
        return {a.x, a.y, b.x, b.y};
    }
    LAT_DEV static void store(char* base, int64_t plane_stride, int64_t s, const mat& m) {
        const uint32_t off = (uint32_t)s * VB;
        const int64_t pb = plane_stride * VB;
        st_plane(base, pb, 0, off, make_double2(m.q0, m.q1));
        st_plane(base, pb, 1, off, make_double2(m.q2, m.q3));
    }
};
struct sq_f32 {  // SU(2), 4 floats: 1 plane of float4
    using vec = float4;  // one plane element
    using real = float;
    using mat = qt<float>;
    static constexpr int NP = 1;
    static constexpr int VB = 16;
    LAT_DEV static mat load(const char* base, int64_t, int64_t s) {
        const float4 a = ld_plane<float4>(base, 0, 0, (uint32_t)s * VB);
        return {a.x, a.y, a.z, a.w};
    }
    LAT_DEV static void store(char* base, int64_t, int64_t s, const mat& m) {
        st_plane(base, 0, 0, (uint32_t)s * VB, make_float4(m.q0, m.q1, m.q2, m.q3));
    }
};

// Address of the first plane of (parity p, direction mu).
template <class ST>
LAT_DEV const char* dir_base(const char* links, int64_t vh_pad, int p, int mu) {
    return links + (int64_t)((p * 4 + mu) * ST::NP) * vh_pad * ST::VB;
}
template <class ST>
LAT_DEV typename ST::mat load_link(const char* links, int64_t vh_pad, int p, int mu, int64_t s) {
    return ST::load(dir_base<ST>(links, vh_pad, p, mu), vh_pad, s);
}
template <class ST>
LAT_DEV typename ST::mat load_link_rows01(const char* links, int64_t vh_pad, int p, int mu, int64_t s) {
    return ST::load_rows01(dir_base<ST>(links, vh_pad, p, mu), vh_pad, s);
}

}  // namespace latdev
