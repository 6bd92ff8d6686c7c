// api_internal.hpp -- host-side pieces shared by the C ABI and the request server.
#pragma once

#include <string>

#include "spkmc_device.hpp"

namespace spkmc {
hipError_t launch_init(const Geom &g, int init, hipStream_t stream);
hipError_t launch_faces(const Geom &g, hipStream_t stream);
hipError_t launch_observables(const Geom &g, hipStream_t stream);
// slab: the per-cycle slab kernels (their counts binned by launch_slab_bin first)
hipError_t launch_cycle(const Geom &g, uint64_t n, uint32_t obs_every, hipStream_t stream, bool slab);
// The per-cycle engine's row kernels (PACKED, octant edge 8 or 16, not RMAX_ALL).
bool rows_supported(const Geom &g);
hipError_t launch_cycle_rows(const Geom &g, uint64_t n, hipStream_t stream);
// Per-cycle slab kernels (PACKED, octant edge 16): the counts of every octant
// once per run, then per cycle the line maximum and the selection with flips.
bool slab_rows_supported(const Geom &g);
hipError_t launch_slab_bin(const Geom &g, hipStream_t stream);
hipError_t launch_cycle_slab(const Geom &g, uint64_t n, hipStream_t stream);
bool persistent_supported(const Geom &g, const spkmc_params &p, bool inc, std::string &why);
hipError_t persistent_configure(const Geom &g, const spkmc_params &p, bool inc, int &grid, int &block,
                                int &wg_domains);
// prep = false skips the slot and flag set-up: allowed only when the previous
// launch on this lattice had the same grid, ended at n0, and the launches since
// the last set-up ran at least two cycles (they then leave the slots and flags
// exactly as the set-up would).
hipError_t launch_persistent(const Geom &g, uint64_t n0, uint64_t ncycles, uint32_t obs_every, int grid,
                             int block, int wg_domains, bool inc, bool prep, hipStream_t stream);
uint64_t persistent_scratch_words(uint64_t K);
// Slab engine (PACKED, octant edge 16, variant 0): support, launch shape, launch.
bool slab_supported(const Geom &g, const spkmc_params &p, std::string &why);
hipError_t slab_configure(const Geom &g, int &grid, int &block, int &wg_domains);
hipError_t launch_slab(const Geom &g, uint64_t n0, uint64_t ncycles, uint32_t obs_every, int grid, bool prep,
                       hipStream_t stream);
struct Replica;
size_t replica_bytes();
// lpd: 1 when every lattice has one line per domain (eight colours) and none
// runs with the fixed bound (a kernel with both fixed at compile time), 0
// otherwise
hipError_t batch_plan(const Geom *const *gs, const uint64_t *n0, const uint64_t *ncycles, uint32_t obs_every,
                      uint32_t n, int P, Replica *out, int &grid, int &block, uint32_t &lpd);
hipError_t upload_replicas(const Replica *host, uint32_t n, Replica *dev, hipStream_t stream);
hipError_t launch_batch(const Replica *dev_reps, uint32_t n, int h, int P, int grid, int block, uint32_t lpd,
                        hipStream_t stream);
hipError_t capture_batch(Replica *dev_reps, uint32_t n, int h, int P, int grid, int block, uint32_t lpd,
                         hipGraph_t *graph);
// The device array of spkmc_run_batch_static on the current device (resolved
// on the first call per device), its capacity in lattices and its bytes.
hipError_t static_replicas(Replica **out);
uint32_t static_replica_cap();
size_t static_replica_bytes();
}  // namespace spkmc

struct spkmc_ctx {
    spkmc_params p;
    hipStream_t stream;
    char *dev;
    size_t dev_bytes;
    spkmc::Geom g;
    size_t spin_off, spin_bytes;   // spin region (A + F, or int8), for save/load
    size_t rec_off;
    uint64_t cycle;                // cycles enqueued
    // the persistent engines' sync words as the last launch left them: ready
    // for a launch of primed_grid workgroups starting at primed_cycle when
    // primed_span (cycles run since their last set-up) is at least 2
    int primed_grid;
    uint64_t primed_cycle, primed_span;
    int engine;
    int grid, block, wg_domains;
    bool failed;
    std::string err;
};

namespace spkmc {
// Workgroups the batch kernel for octant edge h with P passes can keep resident
// at once on the current device (0 on error).
uint32_t batch_capacity(int h, int P, uint32_t lpd = 1);
// Rows (domains per pass) and the most passes of the persistent kernels.
int persist_rows(int h, bool inc);
int persist_max_passes(int h, bool inc);
int batch_max_passes(int h);
uint32_t batch_wgs(const Geom &g, int P);

// The observables of a lattice of N sites with parameters p from a copy of its
// device state header.
void obs_from_state(const spkmc_params &p, uint64_t N, const DevState &st, spkmc_obs *out);
}  // namespace spkmc
