// Host-callable launchers of the kernels in lat_kernels.hip.
#pragma once
#include <hip/hip_runtime.h>

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
// Persistent batch launch (reset counters, work-list kernel, bump the
// members' heat-bath counters).
hipError_t lat_launch_batch(int storage, const BatchArgs& b, uint64_t** counters, int grid, int block,
                            hipStream_t st);
