// Internal interfaces between the host runtime (lbm_capi.hip) and the kernel
// translation units of liblbm.  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_device.h"

namespace lbm {

// Collision operator: BGK (on = 0) or MRT with the given rates of the
// non-viscous moments (the viscous ones relax at 1/tau); s_j <= 0 means
// s_j = 1/tau.
struct MrtParams {
    int on;
    double s_e, s_eps, s_q, s_pi, s_m, s_j;
};

// One flat-interface run of a coexistence launch.
struct CoexCase {
    double *state;  // [19][n] populations, kept between chunks
    double *out;    // rho(n/2), rho(0), largest density change over the chunk, non-finite flag
    double G, tau, rho0, hi, lo;
    MrtParams mrt;
    int init;       // 1: start from the tanh profile between lo and hi
};

// Arguments of one fused step launch over one grid.
// Rows are stored in records of 2^rec_shift rows: a record holds, population
// after population, the segments of its rows ([z][y / k][a][y % k][x] with
// k = 2^rec_shift; k = 1 is row-interleaved [z][y][a][x]).  row_stride is the
// record stride 19 k nx, pop_stride k nx.  Offset of row y within a plane:
__host__ __device__ inline int row_offset(int y, int row_stride, int rec_shift, int nx) {
    return (y >> rec_shift) * row_stride + (y & ((1 << rec_shift) - 1)) * nx;
}

struct StepArgs {
    const void *src;
    void *dst;
    int nx, ny, nz;
    int tiles_x, tiles_y, zchunk, nchunks;
    int tile_w, tile_h;  // tile shape (used by the run-time shaped kernel)
    // element offset of population a at node (x, y, z):
    //   a * pop_stride + z * plane_stride + row_offset(y) + x
    // (the part within a plane fits in 32 bits); see row_offset
    int64_t pop_stride;
    int row_stride, plane_stride, rec_shift;
    double tau, G, rho0, rho_ref;
    MrtParams mrt;
    // Step number of this launch: *step_base + step_add (mod 2^32).  It keys
    // the counter-based random numbers of the stochastic rounding
    // (kStochastic storage kinds); a captured graph replays fixed step_add
    // values over a base the host advances on the device.
    const uint32_t *step_base;
    uint32_t step_add;
};

// One case of a batch: its step arguments (src/dst unset) and both lattices.
struct BatchCase {
    StepArgs args;
    void *lat[2];
};

// Device record of one diagnostics evaluation (mirrors lbm_diag).
struct DiagRecord {
    int64_t step;
    double mass, mom[3], rho_min, rho_max, neck_rho;
    int64_t nonfinite;
};

// Per-block partial of the diagnostics reduction.
struct DiagPartial {
    double mass, mom[3], rho_min, rho_max;
    double nonfinite;
    double pad_;
};

// Description of a lattice for the auxiliary kernels.
struct LatticeRef {
    void *lat;
    int nx, ny, nz;
    int storage;
    int64_t pop_stride;
    int row_stride, plane_stride, rec_shift;
    double rho_ref;
    // Batched cases only: when *frozen != 0 the state lives in pair[*frozen - 1]
    // (the lattice current when the case was frozen) instead of lat.
    const int32_t *frozen;
    void *pair[2];
};

// One component of the droplet labelling (mirrors lbm_droplet).
struct DropletEntry {
    int64_t volume;
    double mass;
    int64_t first_node;
};

// Device arrays of the droplet labelling over n nodes (carved from the
// spare lattice by the host): FP64 density and per-root mass, int32 parent
// and per-root volume, and two int32 counters.
struct DropletScratch {
    double *rho, *mass;
    int32_t *parent, *vol, *counters;
};

struct LigamentArgs {
    int axis;
    double R0, amp_rel, wavelength, c1, c2, width, rho_l, rho_v, noise_amp;
    uint64_t seed;
};

// lbm_step.hip
// Run-time shaped tile of a `threads`-thread workgroup (512 or 1024) for a
// grid: width min(nx, 128 or 256), height balanced over ny with at most
// `threads` nodes and 64 rows per tile.
void dynamic_tile(int threads, int nx, int ny, int *tw, int *th);
int num_tiles();
void tile_shape(int i, int *tx, int *ty);
int find_tile(int tx, int ty);
// A.mrt.on selects the MRT kernel, compiled for the run-time tiles only
// (tile_has_mrt).
hipError_t launch_step(int tile_index, int storage, const StepArgs &A, hipStream_t s);
bool tile_has_mrt(int tile_index);
// Whether this tile's step kernel is compiled for the storage kind (the
// FP32-rest kinds are compiled for the run-time tiles only).
bool tile_has_storage(int tile_index, int storage);
// Workgroups of this tile's step kernel that the device runs at once (compute
// units x resident workgroups per unit); 0 if the runtime cannot say.
int launch_slots(int tile_index, int storage);
hipError_t launch_step_batch(int tile_index, int storage, const BatchCase *cases,
                             const int4 *items, int nitems, const int32_t *frozen, int parity,
                             const uint32_t *step_base, uint32_t step_add, hipStream_t s);

// lbm_aux.hip
hipError_t launch_init_ligament(const LatticeRef &L, const LigamentArgs &g, hipStream_t s);
hipError_t launch_import(const LatticeRef &L, const double *pop, hipStream_t s);
hipError_t launch_export_pop(const LatticeRef &L, double *pop, hipStream_t s);
hipError_t launch_export_rho(const LatticeRef &L, double *rho, hipStream_t s);
hipError_t launch_export_force_u(const LatticeRef &L, const double *rho, double G, double rho0,
                                 double *force, double *u, hipStream_t s);
// Number of partial slots the diagnostics reduction of this grid uses.
int diag_blocks(int nx, int ny, int nz);
// If frozen_flag is given and the state has a non-finite or non-positive
// density, *frozen_flag is set to freeze_value unless it is already set.
hipError_t launch_diag(const LatticeRef &L, int axis, DiagPartial *partials,
                       unsigned long long *slice_max, DiagRecord *out, int64_t step,
                       int32_t *frozen_flag, int32_t freeze_value, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, size_t count, unsigned long long v,
                           hipStream_t s);
// Droplet labelling of the lattice L (6-connected components of rho > rho_mid,
// periodic); leaves the number of components in w.counters[0].
hipError_t launch_droplets_label(const LatticeRef &L, double rho_mid, const DropletScratch &w, hipStream_t s);
// Writes one entry per component (at most cap) into out, in no particular order.
hipError_t launch_droplets_table(const DropletScratch &w, int n, DropletEntry *out, int cap, hipStream_t s);
hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t s);
// One-thread update of a device step counter: *p = v, or *p += v when add.
hipError_t launch_counter(uint32_t *p, uint32_t v, bool add, hipStream_t s);
// Flat-interface coexistence runs, one workgroup each: `chunk` steps on the
// 1 x 1 x n slab held in each case's `state` ([19][n] doubles); init != 0
// first writes the start profile (liquid hi on [n/4, 3n/4), vapour lo
// elsewhere, tanh of width 4).  out[0] = rho(n/2), out[1] = rho(0),
// out[2] = max |rho - rho_before| over the chunk, out[3] = 1 if a non-finite
// density appeared.  The table `cases` is in device memory.
hipError_t launch_coexistence_chunk(const CoexCase *cases, int ncases, int n, int chunk, hipStream_t s);

}  // namespace lbm
