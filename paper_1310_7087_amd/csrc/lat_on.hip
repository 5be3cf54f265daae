// O(N) phi^4 model on one MI355X: an N-vector field on the sites (N = 1..4),
// updated by a checkerboard multi-hit Metropolis sweep, with FP64 reductions
// of <phi^2>, the nearest-neighbour product, <(phi^2-1)^2> and the mean field.
// Kernels and the host side of the lat_on_* calls in include/lat.h.
//
// Layout in HBM: the field is split by parity, then by component, into planes
// of vp = vh rounded up to 256 values (FP64 or FP32): value a of the site with
// half-lattice index s and parity p sits at planes[(p * N + a) * vp + s], so
// every load of a wave is one contiguous run per component.  Generator
// states use the same [parity][word][vp] planes (RANLUX 25 words, MRG32k3a 6).
//
// One thread updates one site: it reads the 2 * 4 neighbours of the other
// parity once, keeps the neighbour sum and the site in registers, and runs
// all NHIT Metropolis hits there, so HBM sees 10 N values per site and pass
// while the arithmetic grows with NHIT (at the paper's NHIT = 100 the pass is
// bound by the vector ALUs: the Philox rounds and the FP64 exponential).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lat.h"
#include "lat_dev.hpp"
#include "lat_hostio.hpp"
#include "lat_launch.hpp"

using namespace latdev;

namespace {

constexpr int ON_BLOCK_MEAS = 256;
constexpr int ON_MEAS_BLOCKS = 1024;  // fixed grid of the measurement: a fixed summation order
constexpr int ON_NOBS = 7;
constexpr int ON_SERIES_CAP = 1024;   // measurements buffered on the device per lat_on_run chunk

struct OnArgs {
    LatGeom g;
    char* field;          // [parity][component][vp] of T
    uint32_t* rl;         // generator states [parity][word][vp] (RANLUX 25, MRG32k3a 6 words), or null
    uint32_t* acc;        // [nblocks] accepted hits of this pass's work-groups
    double kappa, lambda, h, delta, rng_const;
    uint32_t key0, key1, lat_id, sweep;
    int nhit, parity;
};

template <class T>
LAT_DEV T* plane(char* f, int64_t vp, int N, int p, int a) {
    return reinterpret_cast<T*>(f) + ((int64_t)p * N + a) * vp;
}

// Local action s(phi) = -2 kappa F.phi + phi.phi + lambda (phi.phi - 1)^2 - h phi_0,
// evaluated left to right as written (no contraction).
template <int N>
LAT_DEV double local_action(const OnArgs& a, const double (&F)[N], const double (&q)[N]) {
    double fq = 0.0, q2 = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) fq += F[k] * q[k];
#pragma unroll
    for (int k = 0; k < N; ++k) q2 += q[k] * q[k];
    return -2.0 * a.kappa * fq + q2 + a.lambda * (q2 - 1.0) * (q2 - 1.0) - a.h * q[0];
}

// 24-bit uniform from the low bytes of three Philox words (the high 24
// bits of every word feed the proposal)
LAT_DEV double accept_u24(uint32_t w0, uint32_t w1, uint32_t w2) {
    return u24(((w0 & 0xFFu) << 24) | ((w1 & 0xFFu) << 16) | ((w2 & 0xFFu) << 8));
}

template <class T, int N, int RNG>
__global__ void __launch_bounds__(256) on_pass(OnArgs a) {
    __shared__ uint32_t rl_lds[RNG == LAT_RNG_RANLUX_I ? 24 * 256 : 1];
    __shared__ uint32_t wsum[4];
    const int64_t vp = a.g.vh_pad;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int p = a.parity, q = 1 - p;
    uint32_t accepted = 0;
    if (s < a.g.vh) {
        const coord4 c = decode(a.g, s, p);
        int64_t nb[8];
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            nb[2 * mu] = half_index(a.g, step(a.g, c, mu, +1));
            nb[2 * mu + 1] = half_index(a.g, step(a.g, c, mu, -1));
        }
        double F[N], ph[N];
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const T* pl = plane<T>(a.field, vp, N, q, k);
            F[k] = 0.0;
#pragma unroll
            for (int mu = 0; mu < 4; ++mu) F[k] += (double)pl[nb[2 * mu]] + (double)pl[nb[2 * mu + 1]];
            ph[k] = (double)plane<T>(a.field, vp, N, p, k)[s];
        }
        draws<RNG> d;
        uint32_t site = 0;
        mrg_state ms;
        if constexpr (RNG == LAT_RNG_PHILOX_I) {
            site = (uint32_t)canon_index(a.g, c);
        } else if constexpr (RNG == LAT_RNG_MRG_I) {
#pragma unroll
            for (int w = 0; w < 6; ++w) ms.s[w] = a.rl[((int64_t)p * 6 + w) * vp + s];
        } else if constexpr (RNG == LAT_RNG_RANLUX_I) {
            // every site update begins a new block of the site's stream
            uint32_t b[24];
#pragma unroll
            for (int j = 0; j < 24; ++j) b[j] = a.rl[((int64_t)p * 25 + j) * vp + s];
            const uint32_t f = a.rl[((int64_t)p * 25 + 24) * vp + s];
            uint32_t cy = f & 1u;
            ranlux_next_block(b, cy, (f & 2u) == 0);
            d.lds = rl_lds + threadIdx.x;
            d.stride = (int)blockDim.x;
#pragma unroll
            for (int j = 0; j < 24; ++j) d.lds[j * d.stride] = b[j];
            d.c = cy;
            d.idx = 0;
        }
        double s0 = local_action<N>(a, F, ph);
        // delta (2u - 1) for the 24-bit draw v, u = (v + 1/2) 2^-24, is
        // (2v + 1 - 2^24) (delta 2^-24): an exact integer times an exact
        // scale, rounded once, as the plain formula is
        const double dstep = a.delta * (1.0 / 16777216.0);
        for (int k = 0; k < a.nhit; ++k) {
            double tr[N], uacc;
            if constexpr (RNG == LAT_RNG_CONST_I) {
#pragma unroll
                for (int j = 0; j < N; ++j) tr[j] = ph[j] + a.delta * (2.0 * a.rng_const - 1.0);
                uacc = a.rng_const;
            } else {
                uint32_t v[N];
                if constexpr (RNG == LAT_RNG_PHILOX_I) {
                    const u4 o = philox10({site, a.lat_id, a.sweep, (uint32_t)k}, a.key0, a.key1);
                    const uint32_t w[4] = {o.x, o.y, o.z, o.w};
#pragma unroll
                    for (int j = 0; j < N; ++j) v[j] = w[j] >> 8;
                    uacc = accept_u24(o.x, o.y, o.z);
                } else if constexpr (RNG == LAT_RNG_MRG_I) {
#pragma unroll
                    for (int j = 0; j < N; ++j) v[j] = mrg_step(ms) >> 8;
                    uacc = u24(mrg_step(ms));
                } else {
#pragma unroll
                    for (int j = 0; j < N; ++j) v[j] = d.next();
                    uacc = u24(d.next() << 8);
                }
#pragma unroll
                for (int j = 0; j < N; ++j) tr[j] = ph[j] + (double)((int)(2u * v[j] + 1u) - (1 << 24)) * dstep;
            }
            const double s1 = local_action<N>(a, F, tr);
            const double dS = s1 - s0;
            // accept iff uacc < exp(-dS).  exp(-dS) >= 1 > uacc when dS <= 0.
            // Otherwise an FP32 exponential (relative error < 1e-5 for every
            // dS where exp(-dS) can exceed the smallest uacc, 2^-25) decides
            // all but the draws within 1e-4 of the threshold, which take the
            // FP64 exponential: the decision is that of the FP64 test.
            bool acc = true;
            if (dS > 0.0) {
                const double e = (double)__expf((float)(-dS));
                if (uacc > e * (1.0 + 1e-4))
                    acc = false;
                else if (uacc >= e * (1.0 - 1e-4))
                    acc = uacc < exp(-dS);
            }
#pragma unroll
            for (int j = 0; j < N; ++j) ph[j] = acc ? tr[j] : ph[j];
            s0 = acc ? s1 : s0;
            accepted += acc ? 1u : 0u;
        }
#pragma unroll
        for (int k = 0; k < N; ++k) plane<T>(a.field, vp, N, p, k)[s] = (T)ph[k];
        if constexpr (RNG == LAT_RNG_RANLUX_I) {
#pragma unroll
            for (int j = 0; j < 24; ++j) a.rl[((int64_t)p * 25 + j) * vp + s] = d.lds[j * d.stride];
            a.rl[((int64_t)p * 25 + 24) * vp + s] = d.c;  // a block has been delivered
        }
        if constexpr (RNG == LAT_RNG_MRG_I) {
#pragma unroll
            for (int w = 0; w < 6; ++w) a.rl[((int64_t)p * 6 + w) * vp + s] = ms.s[w];
        }
    }
    // accepted hits of the work-group: wave sums, then one store per group
    for (int off = 32; off > 0; off >>= 1) accepted += __shfl_down(accepted, off, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = accepted;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += wsum[w];
        a.acc[blockIdx.x] = t;
    }
}

// Cold (1, 0, ..) or hot (phi_a = 2 u_a - 1) start; RANLUX states seeded on the host.
template <class T, int N, int RNG>
__global__ void __launch_bounds__(256) on_init(OnArgs a, int hot) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t vp = a.g.vh_pad;
    if (j >= 2 * a.g.vh) return;
    const int p = j >= a.g.vh ? 1 : 0;
    const int64_t s = j - p * a.g.vh;
    double u[4] = {0.0, 0.0, 0.0, 0.0};
    if (hot) {
        if constexpr (RNG == LAT_RNG_PHILOX_I) {
            const coord4 c = decode(a.g, s, p);
            const u4 o = philox10({(uint32_t)canon_index(a.g, c), a.lat_id, 0u, 0xFFFFFFFFu}, a.key0, a.key1);
            u[0] = u24(o.x);
            u[1] = u24(o.y);
            u[2] = u24(o.z);
            u[3] = u24(o.w);
        } else if constexpr (RNG == LAT_RNG_RANLUX_I) {
            uint32_t b[24];
            for (int w = 0; w < 24; ++w) b[w] = a.rl[((int64_t)p * 25 + w) * vp + s];
            const uint32_t f = a.rl[((int64_t)p * 25 + 24) * vp + s];
            uint32_t cy = f & 1u;
            ranlux_next_block(b, cy, (f & 2u) == 0);
            for (int k = 0; k < N; ++k) u[k] = u24(b[k] << 8);
            for (int w = 0; w < 24; ++w) a.rl[((int64_t)p * 25 + w) * vp + s] = b[w];
            a.rl[((int64_t)p * 25 + 24) * vp + s] = cy;
        } else if constexpr (RNG == LAT_RNG_MRG_I) {
            mrg_state ms;
            for (int w = 0; w < 6; ++w) ms.s[w] = a.rl[((int64_t)p * 6 + w) * vp + s];
            for (int k = 0; k < N; ++k) u[k] = u24(mrg_step(ms));
            for (int w = 0; w < 6; ++w) a.rl[((int64_t)p * 6 + w) * vp + s] = ms.s[w];
        } else {
            for (int k = 0; k < 4; ++k) u[k] = a.rng_const;
        }
    }
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const double v = hot ? 2.0 * u[k] - 1.0 : (k == 0 ? 1.0 : 0.0);
        plane<T>(a.field, vp, N, p, k)[s] = (T)v;
    }
}

// Per-work-group sums of phi^2, sum_mu phi(x).phi(x+mu), (phi^2-1)^2 and
// phi_a over a fixed grid-stride set of sites; partial[q * nb + block].
template <class T, int N>
__global__ void __launch_bounds__(ON_BLOCK_MEAS) on_meas(OnArgs a, double* partial) {
    __shared__ double red[ON_NOBS][ON_BLOCK_MEAS];
    const int64_t vp = a.g.vh_pad;
    double acc[ON_NOBS] = {0, 0, 0, 0, 0, 0, 0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < 2 * a.g.vh; j += stride) {
        const int p = j >= a.g.vh ? 1 : 0;
        const int64_t s = j - p * a.g.vh;
        const coord4 c = decode(a.g, s, p);
        double ph[N];
#pragma unroll
        for (int k = 0; k < N; ++k) ph[k] = (double)plane<T>(a.field, vp, N, p, k)[s];
        double q2 = 0.0;
#pragma unroll
        for (int k = 0; k < N; ++k) q2 += ph[k] * ph[k];
        double lk = 0.0;
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            const int64_t n = half_index(a.g, step(a.g, c, mu, +1));
            double d = 0.0;
#pragma unroll
            for (int k = 0; k < N; ++k) d += ph[k] * (double)plane<T>(a.field, vp, N, 1 - p, k)[n];
            lk += d;
        }
        acc[0] += q2;
        acc[1] += lk;
        acc[2] += (q2 - 1.0) * (q2 - 1.0);
#pragma unroll
        for (int k = 0; k < N; ++k) acc[3 + k] += ph[k];
    }
#pragma unroll
    for (int o = 0; o < ON_NOBS; ++o) red[o][threadIdx.x] = acc[o];
    __syncthreads();
    for (int w = ON_BLOCK_MEAS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int o = 0; o < ON_NOBS; ++o) red[o][threadIdx.x] += red[o][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < ON_NOBS) partial[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = red[threadIdx.x][0];
}

// Final sums: work-group o adds partial[o][0..nb) with Neumaier compensation
// per thread, then a fixed tree; out[o] = sum / norm(o).
__global__ void __launch_bounds__(256) on_meas_final(const double* partial, int nb, double V, double* out) {
    __shared__ double red[256];
    const int o = blockIdx.x;
    double sum = 0.0, comp = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        const double x = partial[(int64_t)o * nb + b];
        const double t = sum + x;
        comp += fabs(sum) >= fabs(x) ? (sum - t) + x : (x - t) + sum;
        sum = t;
    }
    red[threadIdx.x] = sum + comp;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[o] = red[0] / (o == 1 ? 4.0 * V : V);
}

// canonical [site][component] FP64 <-> device planes
template <class T>
__global__ void __launch_bounds__(256) on_convert(OnArgs a, int N, int to_dev, double* canon) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= 2 * a.g.vh) return;
    const int p = j >= a.g.vh ? 1 : 0;
    const int64_t s = j - p * a.g.vh;
    const int64_t i = canon_index(a.g, decode(a.g, s, p));
    for (int k = 0; k < N; ++k) {
        T* pl = plane<T>(a.field, a.g.vh_pad, N, p, k);
        if (to_dev)
            pl[s] = (T)canon[i * N + k];
        else
            canon[i * N + k] = (double)pl[s];
    }
}

// generator states: device planes [parity][word][vp] <-> canonical [site][nw]
__global__ void __launch_bounds__(256) on_rl_convert(OnArgs a, int nw, int to_dev, uint32_t* canon) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= 2 * a.g.vh) return;
    const int p = j >= a.g.vh ? 1 : 0;
    const int64_t s = j - p * a.g.vh;
    const int64_t i = canon_index(a.g, decode(a.g, s, p));
    for (int w = 0; w < nw; ++w) {
        uint32_t* pl = a.rl + ((int64_t)p * nw + w) * a.g.vh_pad;
        if (to_dev)
            pl[s] = canon[i * nw + w];
        else
            canon[i * nw + w] = pl[s];
    }
}

// ---- dispatch ------------------------------------------------------------
template <class T, int N>
hipError_t launch_pass_t(int rng, const OnArgs& a, int block, hipStream_t st) {
    const dim3 grid((unsigned)((a.g.vh + block - 1) / block));
    switch (rng) {
        case LAT_RNG_PHILOX_I: hipLaunchKernelGGL((on_pass<T, N, LAT_RNG_PHILOX_I>), grid, dim3(block), 0, st, a); break;
        case LAT_RNG_RANLUX_I: hipLaunchKernelGGL((on_pass<T, N, LAT_RNG_RANLUX_I>), grid, dim3(block), 0, st, a); break;
        case LAT_RNG_MRG_I: hipLaunchKernelGGL((on_pass<T, N, LAT_RNG_MRG_I>), grid, dim3(block), 0, st, a); break;
        default: hipLaunchKernelGGL((on_pass<T, N, LAT_RNG_CONST_I>), grid, dim3(block), 0, st, a); break;
    }
    return hipGetLastError();
}
template <class T, int N>
hipError_t launch_init_t(int rng, const OnArgs& a, int hot, hipStream_t st) {
    const dim3 grid((unsigned)((2 * a.g.vh + 255) / 256));
    switch (rng) {
        case LAT_RNG_PHILOX_I: hipLaunchKernelGGL((on_init<T, N, LAT_RNG_PHILOX_I>), grid, dim3(256), 0, st, a, hot); break;
        case LAT_RNG_RANLUX_I: hipLaunchKernelGGL((on_init<T, N, LAT_RNG_RANLUX_I>), grid, dim3(256), 0, st, a, hot); break;
        case LAT_RNG_MRG_I: hipLaunchKernelGGL((on_init<T, N, LAT_RNG_MRG_I>), grid, dim3(256), 0, st, a, hot); break;
        default: hipLaunchKernelGGL((on_init<T, N, LAT_RNG_CONST_I>), grid, dim3(256), 0, st, a, hot); break;
    }
    return hipGetLastError();
}
template <class T, int N>
hipError_t launch_meas_t(const OnArgs& a, int nb, double* partial, hipStream_t st) {
    hipLaunchKernelGGL((on_meas<T, N>), dim3(nb), dim3(ON_BLOCK_MEAS), 0, st, a, partial);
    return hipGetLastError();
}
template <class T>
hipError_t dispatch_n(int N, int what, int rng, const OnArgs& a, int block, int hot, int nb, double* partial,
                      hipStream_t st) {
    switch (N) {
        case 1: return what == 0 ? launch_pass_t<T, 1>(rng, a, block, st) : what == 1 ? launch_init_t<T, 1>(rng, a, hot, st) : launch_meas_t<T, 1>(a, nb, partial, st);
        case 2: return what == 0 ? launch_pass_t<T, 2>(rng, a, block, st) : what == 1 ? launch_init_t<T, 2>(rng, a, hot, st) : launch_meas_t<T, 2>(a, nb, partial, st);
        case 3: return what == 0 ? launch_pass_t<T, 3>(rng, a, block, st) : what == 1 ? launch_init_t<T, 3>(rng, a, hot, st) : launch_meas_t<T, 3>(a, nb, partial, st);
        default: return what == 0 ? launch_pass_t<T, 4>(rng, a, block, st) : what == 1 ? launch_init_t<T, 4>(rng, a, hot, st) : launch_meas_t<T, 4>(a, nb, partial, st);
    }
}

std::string hip_msg(const char* what, hipError_t e) { return std::string(what) + " failed: " + hipGetErrorString(e); }

}  // namespace

// ---- host side ---------------------------------------------------------------
struct lat_on_ctx {
    int n = 4, storage = LAT_F64, rng = LAT_RNG_PHILOX, start = LAT_HOT, nhit = 100, block = 256;
    double kappa = 0, lambda = 0, h = 0, delta = 1, rng_const = 0.5;
    uint64_t seed = 0, sweeps = 0;
    uint32_t lat_id = 0;
    LatGeom g{};
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char* base = nullptr;
    bool own_mem = false;
    size_t field_off = 0, rl_off = 0, acc_off = 0, part_off = 0, series_off = 0, total = 0;
    size_t rl_bytes = 0;
    int nb_pass = 0;

    char* field() const { return base + field_off; }
    uint32_t* rl() const { return rl_bytes ? reinterpret_cast<uint32_t*>(base + rl_off) : nullptr; }
    uint32_t* acc(int p) const { return reinterpret_cast<uint32_t*>(base + acc_off) + (size_t)p * nb_pass; }
    double* partial() const { return reinterpret_cast<double*>(base + part_off); }
    double* series() const { return reinterpret_cast<double*>(base + series_off); }
    int64_t V() const { return 2 * g.vh; }
};

namespace {

#define ON_TRY(expr)                                                   \
    do {                                                               \
        hipError_t e_ = (expr);                                        \
        if (e_ != hipSuccess) return lat_internal_fail(LAT_EDEVICE, hip_msg(#expr, e_).c_str()); \
    } while (0)

size_t up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// 32-bit words of per-site generator state
int state_words(int rng) { return rng == LAT_RNG_RANLUX ? 25 : rng == LAT_RNG_MRG32K3A ? 6 : 0; }

// Parameter checks and the device layout; 0 on success.
int on_layout(lat_on_ctx& c, int n, const int d[4], const lat_options& o) {
    if (n < 1 || n > 4) return lat_internal_fail(LAT_EINVAL, "O(N): ncomp must be 1..4");
    for (int k = 0; k < 4; ++k)
        if (d[k] < 2 || d[k] % 2) return lat_internal_fail(LAT_EINVAL, "extents must be even and >= 2");
    const int64_t V = (int64_t)d[0] * d[1] * d[2] * d[3];
    if (V > ((int64_t)1 << 32)) return lat_internal_fail(LAT_EINVAL, "lattice too large (V > 2^32)");
    if (o.storage != LAT_F64 && o.storage != LAT_F32)
        return lat_internal_fail(LAT_EUNSUPPORTED, "O(N) fields are stored as LAT_F64 or LAT_F32");
    if (o.rng < LAT_RNG_MRG32K3A || o.rng > LAT_RNG_RANLUX) return lat_internal_fail(LAT_EINVAL, "unknown generator");
    if (o.rng == LAT_RNG_CONST && !(o.rng_const > 0.0 && o.rng_const < 1.0))
        return lat_internal_fail(LAT_EINVAL, "rng_const must lie in (0,1)");
    if (o.nhit < 1 || o.nhit > 1000) return lat_internal_fail(LAT_EINVAL, "O(N): nhit must be 1..1000");
    if (o.start != LAT_COLD && o.start != LAT_HOT) return lat_internal_fail(LAT_EINVAL, "bad start");
    if (o.frozen != LAT_FROZEN_NONE) return lat_internal_fail(LAT_EUNSUPPORTED, "frozen links are an SU(N) option");
    if (o.block_size != 0 && o.block_size != 64 && o.block_size != 128 && o.block_size != 256)
        return lat_internal_fail(LAT_EINVAL, "block_size must be 0, 64, 128 or 256");
    c.n = n;
    c.storage = o.storage;
    c.rng = o.rng;
    c.block = o.block_size ? o.block_size : 256;
    c.g.nx = d[0];
    c.g.ny = d[1];
    c.g.nz = d[2];
    c.g.nt = d[3];
    c.g.nxh = d[0] / 2;
    c.g.vh = V / 2;
    c.g.vh_pad = (int64_t)up((size_t)c.g.vh, 256);
    const size_t tb = o.storage == LAT_F64 ? 8 : 4;
    c.nb_pass = (int)((c.g.vh + 63) / 64);  // enough slots for the smallest work-group size
    size_t off = 0;
    c.field_off = off;
    off = up(off + 2 * (size_t)n * c.g.vh_pad * tb, 256);
    c.rl_off = off;
    c.rl_bytes = 2 * (size_t)state_words(o.rng) * c.g.vh_pad * 4;
    off = up(off + c.rl_bytes, 256);
    c.acc_off = off;
    off = up(off + 2 * (size_t)c.nb_pass * 4, 256);
    c.part_off = off;
    off = up(off + (size_t)ON_NOBS * ON_MEAS_BLOCKS * 8, 256);
    c.series_off = off;
    off = up(off + (size_t)ON_NOBS * ON_SERIES_CAP * 8, 256);
    c.total = off;
    return LAT_OK;
}

OnArgs on_args(const lat_on_ctx* c, int parity) {
    OnArgs a{};
    a.g = c->g;
    a.field = c->field();
    a.rl = c->rl();
    a.acc = c->acc(parity);
    a.kappa = c->kappa;
    a.lambda = c->lambda;
    a.h = c->h;
    a.delta = c->delta;
    a.rng_const = c->rng_const;
    a.key0 = (uint32_t)c->seed;
    a.key1 = (uint32_t)(c->seed >> 32);
    a.lat_id = c->lat_id;
    a.sweep = (uint32_t)c->sweeps;
    a.nhit = c->nhit;
    a.parity = parity;
    return a;
}

int rng_i(int rng) {
    return rng == LAT_RNG_PHILOX ? LAT_RNG_PHILOX_I
           : rng == LAT_RNG_RANLUX ? LAT_RNG_RANLUX_I
           : rng == LAT_RNG_MRG32K3A ? LAT_RNG_MRG_I
                                     : LAT_RNG_CONST_I;
}

hipError_t launch(const lat_on_ctx* c, int what, const OnArgs& a, int hot, double* partial) {
    if (c->storage == LAT_F64)
        return dispatch_n<double>(c->n, what, rng_i(c->rng), a, c->block, hot, ON_MEAS_BLOCKS, partial, c->stream);
    return dispatch_n<float>(c->n, what, rng_i(c->rng), a, c->block, hot, ON_MEAS_BLOCKS, partial, c->stream);
}

// Queues one sweep: parity 0 then parity 1.
int enqueue_sweep(lat_on_ctx* c) {
    for (int p = 0; p < 2; ++p) ON_TRY(launch(c, 0, on_args(c, p), 0, nullptr));
    c->sweeps += 1;
    return LAT_OK;
}

int enqueue_measure(lat_on_ctx* c, double* out) {
    ON_TRY(launch(c, 2, on_args(c, 0), 0, c->partial()));
    hipLaunchKernelGGL(on_meas_final, dim3(ON_NOBS), dim3(256), 0, c->stream, (const double*)c->partial(),
                       ON_MEAS_BLOCKS, (double)c->V(), out);
    ON_TRY(hipGetLastError());
    return LAT_OK;
}

// Per-site generator states on the host, canonical site order: RANLUX 25
// words (seeded as the SU(N) streams are), MRG32k3a 6 words (streams 2^127
// apart).
std::vector<uint32_t> canonical_states(const lat_on_ctx* c) {
    if (c->rng == LAT_RNG_MRG32K3A) return lat_internal_mrg_site_states(c->seed, c->V());
    const uint64_t M = 2147483561ull;
    std::vector<uint32_t> out((size_t)c->V() * 25);
    for (int64_t i = 0; i < c->V(); ++i) {
        const uint64_t j = ((uint64_t)i + 2654435761ull * (uint64_t)c->lat_id) % M;
        uint64_t e = 1 + ((c->seed % M) + 1000003ull * j) % M;
        uint32_t* w = &out[(size_t)i * 25];
        for (int k = 0; k < 24; ++k) {
            e = (40014ull * e) % 2147483563ull;
            w[k] = (uint32_t)(e & 0xFFFFFFu);
        }
        w[24] = (w[23] == 0 ? 1u : 0u) | 2u;
    }
    return out;
}

// Copies the generator states between the device planes and a host array in
// canonical site order; synchronises.
int rl_transfer(lat_on_ctx* c, uint32_t* host, bool to_dev) {
    const int nw = state_words(c->rng);
    const size_t n = (size_t)c->V() * nw;
    uint32_t* dev = nullptr;
    ON_TRY(hipMalloc((void**)&dev, n * 4));
    hipError_t e = hipSuccess;
    if (to_dev) e = hipMemcpyAsync(dev, host, n * 4, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(on_rl_convert, dim3((unsigned)((c->V() + 255) / 256)), dim3(256), 0, c->stream,
                           on_args(c, 0), nw, to_dev ? 1 : 0, dev);
        e = hipGetLastError();
    }
    if (e == hipSuccess && !to_dev) e = hipMemcpyAsync(host, dev, n * 4, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(dev);
    if (e != hipSuccess) return lat_internal_fail(LAT_EDEVICE, hip_msg("generator state transfer", e).c_str());
    return LAT_OK;
}

void destroy(lat_on_ctx* c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    if (c->own_mem && c->base) (void)hipFree(c->base);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

int create_device(lat_on_ctx* c, const lat_options& o) {
    ON_TRY(hipGetDevice(&c->device));
    if (o.stream) {
        c->stream = (hipStream_t)o.stream;
    } else {
        ON_TRY(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
        c->own_stream = true;
    }
    if (o.device_buffer) {
        if (o.device_bytes < c->total) return lat_internal_fail(LAT_ENOMEM, "caller device buffer too small");
        if (((uintptr_t)o.device_buffer) & 255) return lat_internal_fail(LAT_EINVAL, "device_buffer must be 256-byte aligned");
        c->base = (char*)o.device_buffer;
    } else {
        if (hipMalloc((void**)&c->base, c->total) != hipSuccess) {
            c->base = nullptr;
            (void)hipGetLastError();
            return lat_internal_fail(LAT_ENOMEM, "hipMalloc of the O(N) field failed");
        }
        c->own_mem = true;
    }
    ON_TRY(hipMemsetAsync(c->base, 0, c->total, c->stream));
    if (state_words(c->rng)) {
        std::vector<uint32_t> st = canonical_states(c);
        const int rc = rl_transfer(c, st.data(), true);
        if (rc) return rc;
    }
    ON_TRY(launch(c, 1, on_args(c, 0), c->start == LAT_HOT, nullptr));
    return LAT_OK;
}

}  // namespace

extern "C" {

size_t lat_on_device_bytes(int ncomp, int Nx, int Ny, int Nz, int Nt, const lat_options* opt) {
    lat_options o;
    lat_default_options(&o);
    o.nhit = 100;
    if (opt) o = *opt;
    lat_on_ctx c;
    const int d[4] = {Nx, Ny, Nz, Nt};
    if (on_layout(c, ncomp, d, o) != LAT_OK) return 0;
    return c.total;
}

int lat_on_create(lat_on_t* out, int ncomp, int Nx, int Ny, int Nz, int Nt, double kappa, double lambda,
                  double h, double delta, const lat_options* opt) {
    if (!out) return lat_internal_fail(LAT_EINVAL, "NULL output handle");
    *out = nullptr;
    lat_options o;
    lat_default_options(&o);
    o.nhit = 100;
    if (opt) o = *opt;
    if (!std::isfinite(kappa) || !std::isfinite(lambda) || !(lambda >= 0.0) || !std::isfinite(h) ||
        !(delta > 0.0) || !std::isfinite(delta))
        return lat_internal_fail(LAT_EINVAL, "O(N): kappa and h finite, lambda >= 0, delta > 0 required");
    lat_on_ctx* c = new lat_on_ctx();
    const int d[4] = {Nx, Ny, Nz, Nt};
    int rc = on_layout(*c, ncomp, d, o);
    if (rc) {
        delete c;
        return rc;
    }
    c->kappa = kappa;
    c->lambda = lambda;
    c->h = h;
    c->delta = delta;
    c->rng_const = o.rng_const;
    c->start = o.start;
    c->nhit = o.nhit;
    c->lat_id = o.lattice_id;
    const uint64_t MRG_M2 = 4294944443ull;
    uint64_t seed = o.seed;
    if (seed == 0) {
        seed = (uint64_t)std::chrono::high_resolution_clock::now().time_since_epoch().count();
        seed ^= seed >> 29;
        if (!seed) seed = 1;
        if (o.rng == LAT_RNG_MRG32K3A) seed = 1 + seed % (MRG_M2 - 1);
    }
    if (o.rng == LAT_RNG_MRG32K3A && seed >= MRG_M2) {
        delete c;
        return lat_internal_fail(LAT_EINVAL, "MRG32k3a seed must be in [1, 4294944443)");
    }
    c->seed = seed;
    rc = create_device(c, o);
    if (rc) {
        std::string keep = lat_last_error();
        destroy(c);
        lat_internal_fail(rc, keep.c_str());
        return rc;
    }
    *out = c;
    return LAT_OK;
}

int lat_on_sweep(lat_on_t c, int n_sweeps) {
    if (!c) return lat_internal_fail(LAT_EINVAL, "NULL handle");
    if (n_sweeps < 0) return lat_internal_fail(LAT_EINVAL, "negative sweep count");
    for (int k = 0; k < n_sweeps; ++k) {
        int rc = enqueue_sweep(c);
        if (rc) return rc;
    }
    return LAT_OK;
}

int lat_on_measure(lat_on_t c, double obs[7]) {
    if (!c || !obs) return lat_internal_fail(LAT_EINVAL, "NULL argument");
    int rc = enqueue_measure(c, c->series());
    if (rc) return rc;
    ON_TRY(hipMemcpyAsync(obs, c->series(), ON_NOBS * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    ON_TRY(hipStreamSynchronize(c->stream));
    return LAT_OK;
}

int lat_on_run(lat_on_t c, int n_sweeps, int measure_every, double* series) {
    if (!c) return lat_internal_fail(LAT_EINVAL, "NULL handle");
    if (n_sweeps < 0 || measure_every < 0) return lat_internal_fail(LAT_EINVAL, "negative argument");
    int pending = 0, done = 0;
    auto flush = [&]() -> int {
        if (pending && series)
            ON_TRY(hipMemcpyAsync(series + (size_t)ON_NOBS * done, c->series(), (size_t)pending * ON_NOBS * sizeof(double),
                                  hipMemcpyDeviceToHost, c->stream));
        ON_TRY(hipStreamSynchronize(c->stream));
        done += pending;
        pending = 0;
        return LAT_OK;
    };
    for (int k = 1; k <= n_sweeps; ++k) {
        int rc = enqueue_sweep(c);
        if (rc) return rc;
        if (measure_every > 0 && k % measure_every == 0) {
            rc = enqueue_measure(c, c->series() + (size_t)ON_NOBS * pending);
            if (rc) return rc;
            if (++pending == ON_SERIES_CAP && (rc = flush())) return rc;
        }
    }
    return flush();
}

int lat_on_acceptance(lat_on_t c, double* rate) {
    if (!c || !rate) return lat_internal_fail(LAT_EINVAL, "NULL argument");
    if (c->sweeps == 0) return lat_internal_fail(LAT_ESTATE, "no sweep has run yet");
    const int nb = (int)((c->g.vh + c->block - 1) / c->block);
    std::vector<uint32_t> a((size_t)2 * c->nb_pass);
    ON_TRY(hipMemcpyAsync(a.data(), c->acc(0), a.size() * 4, hipMemcpyDeviceToHost, c->stream));
    ON_TRY(hipStreamSynchronize(c->stream));
    uint64_t t = 0;
    for (int p = 0; p < 2; ++p)
        for (int b = 0; b < nb; ++b) t += a[(size_t)p * c->nb_pass + b];
    *rate = (double)t / ((double)c->V() * (double)c->nhit);
    return LAT_OK;
}

int lat_on_get_field(lat_on_t c, double* host, size_t n) {
    if (!c || !host) return lat_internal_fail(LAT_EINVAL, "NULL argument");
    if (n != (size_t)c->V() * c->n) return lat_internal_fail(LAT_EINVAL, "buffer must hold V * N doubles");
    double* dev = nullptr;
    ON_TRY(hipMalloc((void**)&dev, n * sizeof(double)));
    OnArgs a = on_args(c, 0);
    const dim3 grid((unsigned)((c->V() + 255) / 256));
    if (c->storage == LAT_F64)
        hipLaunchKernelGGL(on_convert<double>, grid, dim3(256), 0, c->stream, a, c->n, 0, dev);
    else
        hipLaunchKernelGGL(on_convert<float>, grid, dim3(256), 0, c->stream, a, c->n, 0, dev);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(host, dev, n * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(dev);
    if (e != hipSuccess) return lat_internal_fail(LAT_EDEVICE, hip_msg("lat_on_get_field", e).c_str());
    return LAT_OK;
}

int lat_on_set_field(lat_on_t c, const double* host, size_t n) {
    if (!c || !host) return lat_internal_fail(LAT_EINVAL, "NULL argument");
    if (n != (size_t)c->V() * c->n) return lat_internal_fail(LAT_EINVAL, "buffer must hold V * N doubles");
    double* dev = nullptr;
    ON_TRY(hipMalloc((void**)&dev, n * sizeof(double)));
    hipError_t e = hipMemcpyAsync(dev, host, n * sizeof(double), hipMemcpyHostToDevice, c->stream);
    OnArgs a = on_args(c, 0);
    const dim3 grid((unsigned)((c->V() + 255) / 256));
    if (e == hipSuccess) {
        if (c->storage == LAT_F64)
            hipLaunchKernelGGL(on_convert<double>, grid, dim3(256), 0, c->stream, a, c->n, 1, dev);
        else
            hipLaunchKernelGGL(on_convert<float>, grid, dim3(256), 0, c->stream, a, c->n, 1, dev);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(dev);
    if (e != hipSuccess) return lat_internal_fail(LAT_EDEVICE, hip_msg("lat_on_set_field", e).c_str());
    return LAT_OK;
}

int lat_on_get_info(lat_on_t c, uint64_t* seed_used, uint64_t* sweeps_done) {
    if (!c) return lat_internal_fail(LAT_EINVAL, "NULL handle");
    if (seed_used) *seed_used = c->seed;
    if (sweeps_done) *sweeps_done = c->sweeps;
    return LAT_OK;
}

int lat_on_profile(lat_on_t c, int reps, double* ms_per_pass) {
    if (!c || !ms_per_pass || reps < 1) return lat_internal_fail(LAT_EINVAL, "NULL argument or reps < 1");
    hipEvent_t e0, e1;
    ON_TRY(hipEventCreate(&e0));
    hipError_t e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        return lat_internal_fail(LAT_EDEVICE, hip_msg("hipEventCreate", e).c_str());
    }
    int rc = LAT_OK;
    float ms = 0.0f;
    e = hipEventRecord(e0, c->stream);
    for (int k = 0; k < reps && e == hipSuccess && rc == LAT_OK; ++k) rc = enqueue_sweep(c);
    if (e == hipSuccess && rc == LAT_OK) e = hipEventRecord(e1, c->stream);
    if (e == hipSuccess && rc == LAT_OK) e = hipEventSynchronize(e1);
    if (e == hipSuccess && rc == LAT_OK) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (e != hipSuccess) return lat_internal_fail(LAT_EDEVICE, hip_msg("lat_on_profile", e).c_str());
    *ms_per_pass = (double)ms / (2.0 * reps);
    return LAT_OK;
}

int lat_on_save(lat_on_t c, const char* path) {
    if (!c || !path) return lat_internal_fail(LAT_EINVAL, "NULL argument");
    std::vector<double> field((size_t)c->V() * c->n);
    int rc = lat_on_get_field(c, field.data(), field.size());
    if (rc) return rc;
    std::vector<uint32_t> words;
    if (state_words(c->rng)) {
        words.resize((size_t)c->V() * state_words(c->rng));
        if ((rc = rl_transfer(c, words.data(), false))) return rc;
    }
    lathost::on_header hd;
    lathost::on_header_init(hd);
    hd.ncomp = (uint32_t)c->n;
    hd.dims[0] = (uint32_t)c->g.nx;
    hd.dims[1] = (uint32_t)c->g.ny;
    hd.dims[2] = (uint32_t)c->g.nz;
    hd.dims[3] = (uint32_t)c->g.nt;
    hd.storage = (uint32_t)c->storage;
    hd.rng = (uint32_t)c->rng;
    hd.start = (uint32_t)c->start;
    hd.nhit = (uint32_t)c->nhit;
    hd.lat_id = c->lat_id;
    hd.kappa = c->kappa;
    hd.lambda = c->lambda;
    hd.h = c->h;
    hd.delta = c->delta;
    hd.rng_const = c->rng_const;
    hd.seed = c->seed;
    hd.sweeps = c->sweeps;
    hd.n_doubles = field.size();
    hd.n_words = words.size();
    if (!lathost::write_checkpoint(path, &hd, sizeof hd, field.data(), field.size(), words.data(), words.size()))
        return lat_internal_fail(LAT_EIO, (std::string("write of ") + path + " failed").c_str());
    return LAT_OK;
}

int lat_on_load(lat_on_t* out, const char* path, const lat_options* opt) {
    if (!out || !path) return lat_internal_fail(LAT_EINVAL, "NULL argument");
    *out = nullptr;
    lathost::on_header hd;
    std::vector<double> field;
    std::vector<uint32_t> words;
    switch (lathost::read_on_checkpoint(path, hd, field, words)) {
        case lathost::CKPT_OK: break;
        case lathost::CKPT_CANNOT_OPEN: return lat_internal_fail(LAT_EIO, (std::string("cannot open ") + path).c_str());
        case lathost::CKPT_BAD_HEADER: return lat_internal_fail(LAT_ECORRUPT, "not an O(N) checkpoint (or its header is inconsistent)");
        case lathost::CKPT_BAD_SIZE: return lat_internal_fail(LAT_ECORRUPT, "O(N) checkpoint is truncated or has trailing data");
        case lathost::CKPT_NO_MEMORY: return lat_internal_fail(LAT_ENOMEM, "no host memory for the O(N) checkpoint");
        default: return lat_internal_fail(LAT_ECORRUPT, "O(N) checkpoint checksum mismatch");
    }
    lat_options o;
    lat_default_options(&o);
    if (opt) o = *opt;
    else o.storage = (int)hd.storage;
    o.rng = (int)hd.rng;
    o.rng_const = hd.rng_const;
    o.start = LAT_COLD;  // replaced below
    o.seed = hd.seed;
    o.nhit = (int)hd.nhit;
    o.lattice_id = hd.lat_id;
    lat_on_t c = nullptr;
    int rc = lat_on_create(&c, (int)hd.ncomp, (int)hd.dims[0], (int)hd.dims[1], (int)hd.dims[2], (int)hd.dims[3],
                           hd.kappa, hd.lambda, hd.h, hd.delta, &o);
    if (rc) return rc;
    c->start = (int)hd.start;
    c->sweeps = hd.sweeps;
    rc = lat_on_set_field(c, field.data(), field.size());
    if (!rc && !words.empty()) rc = rl_transfer(c, words.data(), true);
    if (rc) {
        const std::string keep = lat_last_error();
        destroy(c);
        return lat_internal_fail(rc, keep.c_str());
    }
    *out = c;
    return LAT_OK;
}

int lat_on_destroy(lat_on_t c) {
    destroy(c);
    return LAT_OK;
}

}  // extern "C"
