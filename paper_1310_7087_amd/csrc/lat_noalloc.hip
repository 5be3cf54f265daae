// Link read-out without device allocation, for callers that cannot allocate
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc).  The canonical FP64 links pass through one fixed device array
// per GPU, `scratch`, in chunks of whole sites; each chunk is converted by a
// kernel and copied to the caller's host buffer before the next one starts
// (both on the handle's stream, so stream order keeps them apart).
//
// `scratch` is a file-scope __device__ array: every GPU the library runs on
// holds its own copy, at its own address, until the process ends.  Host code
// never passes the array's name to a kernel or a copy (on the host it is only
// a stand-in symbol); it asks the runtime for the device address once per
// device, with that device current, and uses that address from then on.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/lat.h"
#include "lat_dev.hpp"
#include "lat_launch.hpp"

using namespace latdev;

namespace {

static __device__ __align__(256) char scratch[LAT_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_ptr[MAX_DEVICES] = {};

// Canonical sites [i0, i0 + n) of the lattice -> out[(i - i0) * 4 + mu][comp]
// (the same loads and conversions as the whole-lattice read-out).
template <class ST, int NG>
__global__ void __launch_bounds__(256) to_canonical_range(LatGeom g, const char* links, int64_t i0, int64_t n,
                                                          double* out) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int64_t i = i0 + j;
    coord4 c;
    int64_t r = i;
    c.x = (int)(r % g.nx);
    r /= g.nx;
    c.y = (int)(r % g.ny);
    r /= g.ny;
    c.z = (int)(r % g.nz);
    c.t = (int)(r / g.nz);
    const int p = (c.x + c.y + c.z + c.t) & 1;
    const int64_t s = half_index(g, c);
    for (int mu = 0; mu < 4; ++mu) {
        const typename ST::mat m = load_link<ST>(links, g.vh_pad, p, mu, s);
        if constexpr (NG == 3) {
            double* dst = out + (j * 4 + mu) * 18;
            for (int k = 0; k < 9; ++k) {
                dst[2 * k] = (double)m.e[k / 3][k % 3].re;
                dst[2 * k + 1] = (double)m.e[k / 3][k % 3].im;
            }
        } else {
            double* dst = out + (j * 4 + mu) * 4;
            dst[0] = (double)m.q0;
            dst[1] = (double)m.q1;
            dst[2] = (double)m.q2;
            dst[3] = (double)m.q3;
        }
    }
}

template <class ST, int NG>
hipError_t launch_range(const LatGeom& g, const char* links, int64_t i0, int64_t n, double* out, hipStream_t st) {
    hipLaunchKernelGGL((to_canonical_range<ST, NG>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, links,
                       i0, n, out);
    return hipGetLastError();
}

hipError_t launch_range_any(int group, int storage, const LatGeom& g, const char* links, int64_t i0, int64_t n,
                            double* out, hipStream_t st) {
    if (group == 3) {
        switch (storage) {
            case LAT_ST_F64: return launch_range<st_f64, 3>(g, links, i0, n, out, st);
            case LAT_ST_F32: return launch_range<st_f32, 3>(g, links, i0, n, out, st);
            case LAT_ST_F64C12: return launch_range<st_f64c12, 3>(g, links, i0, n, out, st);
            default: return launch_range<st_f32c12, 3>(g, links, i0, n, out, st);
        }
    }
    if (storage == LAT_ST_F64) return launch_range<sq_f64, 2>(g, links, i0, n, out, st);
    return launch_range<sq_f32, 2>(g, links, i0, n, out, st);
}

// Device address of this device's `scratch`, looked up once per device with
// that device current (the caller's current device).
hipError_t scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

}  // namespace

hipError_t lat_noalloc_get_links(int group, int storage, const LatGeom& g, const char* links, double* host,
                                 hipStream_t st) {
    void* base = nullptr;
    hipError_t e = scratch_address(&base);
    if (e != hipSuccess) return e;
    const int64_t per_site = 4LL * (group == 3 ? 18 : 4);  // doubles
    const int64_t chunk = (int64_t)(LAT_NOALLOC_SCRATCH_BYTES / sizeof(double)) / per_site;
    const int64_t V = 2 * g.vh;
    double* buf = static_cast<double*>(base);
    for (int64_t i0 = 0; i0 < V; i0 += chunk) {
        const int64_t n = V - i0 < chunk ? V - i0 : chunk;
        e = launch_range_any(group, storage, g, links, i0, n, buf, st);
        if (e != hipSuccess) return e;
        // the copy is ordered after the kernel and before the next chunk's
        // kernel on the same stream
        e = hipMemcpyAsync(host + i0 * per_site, buf, (size_t)(n * per_site) * sizeof(double), hipMemcpyDeviceToHost,
                           st);
        if (e != hipSuccess) return e;
    }
    return hipStreamSynchronize(st);
}
