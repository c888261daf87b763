// Layout of the per-device scratch array of tp_bin_noalloc (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tp_kernel.h"

namespace tpk {

// Limits of one allocation-free call: events (every event of a call may need
// the later tiers, so the deferral list holds one entry per event) and edge
// doubles (the edge data of both axes, see edge_doubles()).
constexpr int64_t NA_MAX_EVENTS = int64_t(1) << 22;
constexpr int NA_EDGES = 384;

constexpr size_t NA_SAMPLE_OFF = 0;                                  // KSample
constexpr size_t NA_COUNT_OFF = 512;                                 // list count, finished workgroups
constexpr size_t NA_EDGES_OFF = 1024;                                // doubles[NA_EDGES]
constexpr size_t NA_LIST_OFF = 4096;                                 // uint64[NA_MAX_EVENTS]
constexpr size_t NA_BYTES = NA_LIST_OFF + size_t(NA_MAX_EVENTS) * 8; // 32 MiB + 4 KiB
static_assert(sizeof(KSample) <= NA_COUNT_OFF - NA_SAMPLE_OFF, "descriptor slot too small");
static_assert(NA_EDGES_OFF + NA_EDGES * 8 <= NA_LIST_OFF, "edge slot too small");

// Device address of this device's scratch array (taken once per device).
hipError_t noalloc_scratch(int device, unsigned char **out);
// Enqueue the set-up kernel: descriptor and edges into the array, counters cleared.
hipError_t launch_noalloc_setup(const KSample &k, const double *edges, int nedges, unsigned char *base,
                                hipStream_t st);

}  // namespace tpk
