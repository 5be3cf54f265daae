// Host-callable launchers of the kernels in lat_kernels.hip.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "lat_types.hpp"

hipError_t lat_launch_pass(int group, int storage, int kind, bool reunit, int rng, const PassArgs& a, int block,
                           hipStream_t st);
hipError_t lat_launch_init(int group, int storage, int rng, const InitArgs& a, hipStream_t st);
hipError_t lat_launch_measure(int group, int storage, const MeasArgs& a, double* out, uint32_t* slot_counter,
                              hipStream_t st);
hipError_t lat_launch_convert(int group, int storage, bool to_dev, const LatGeom& g, double* canon, char* links,
                              hipStream_t st);
hipError_t lat_launch_bump(uint64_t* counter, int n, hipStream_t st);
hipError_t lat_launch_philox(const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t* out, int64_t n,
                             hipStream_t st);
// Batch launch of n_sweeps compound sweeps: mode 0 = one kernel per pass over
// all members, mode 1 = one persistent work-list kernel; then the members'
// heat-bath counters are advanced.
hipError_t lat_launch_batch(int storage, int mode, const BatchArgs& b, uint64_t** counters, int grid, int block,
                            hipStream_t st);
// Canonical FP64 links of a lattice copied to host memory through this
// device's fixed scratch array, chunk by chunk (no allocation); synchronises.
hipError_t lat_noalloc_get_links(int group, int storage, const LatGeom& g, const char* links, double* host,
                                 hipStream_t st);
// Sets the calling thread's error message (lat_last_error) and returns code.
int lat_internal_fail(int code, const char* msg);
// MRG32k3a states of sites 0..nsites-1 (6 words each): the seed's stream
// (s, s, s, s, s, s) advanced by 2^127 steps per site.
std::vector<uint32_t> lat_internal_mrg_site_states(uint64_t seed, int64_t nsites);
