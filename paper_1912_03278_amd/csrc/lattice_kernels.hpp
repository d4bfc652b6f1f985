// Launch interface of the fused lattice passes (lattice_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "ihmc_internal.hpp"

namespace ihmc {

// PASS_PAIR: the middle steps j and j + 1 in one launch (2D tile classes only).
enum PassMode : int { PASS_FIRST = 0, PASS_MIDDLE = 1, PASS_LAST = 2, PASS_MEASURE = 3, PASS_FORCE = 4, PASS_PAIR = 5 };

struct TileShape {
  int bx, by, bz;
};

// Built-in tile class of a lattice (row length L0, planes L2; L2 = 1 in 2D):
// the class that the context uses unless its tuning table has an entry for it.
int tile_class(int ndim, int L0, int L2);

// Number of tile classes of a dimension (2 or 3); classes are 0 .. n-1.
int tile_class_count(int ndim);

// Tile extents used for a state precision (4 or 8 bytes), dimension (2 or 3)
// and tile class.
TileShape tile_shape(int precision, int ndim, int cls);

// Chains small enough for one workgroup's LDS run whole trajectories per launch
// (lattice_resident): their launch group has this tile class, and one Tile
// entry per chain.
constexpr int RESIDENT_CLASS = -1;
// Chains of the inverse (phi) formulation run whole trajectories per launch
// too (lattice_resident_phi, FP64): their own launch group.
constexpr int RESIDENT_PHI_CLASS = -2;
// Largest phi-form chain (sites) that fits one workgroup's LDS.
int resident_phi_max_sites(bool site_field);
hipError_t launch_lattice_resident_phi(int ndim, const ChainDev* chains, const Tile* tiles, int n_chains, int n_traj,
                                       hipStream_t s);
// Largest chain (sites) of a state precision (4 or 8 bytes) that fits, with or
// without a per-site field.
int resident_max_sites(int precision, bool site_field);
// n_traj trajectories of each of n_chains resident chains (tiles[b].chain is
// block b's chain); n_traj = 0 measures S and the estimator sums instead.
// per_cu: chains a CU may hold at once, 2 (the kernel's LDS and register
// budget) or 1 (the launch runs beside tiled passes, which keep the rest of
// the CU's LDS).
hipError_t launch_lattice_resident(int precision, int ndim, const ChainDev* chains, const Tile* tiles, int n_chains,
                                   int n_traj, int per_cu, hipStream_t s);

// Launch one pass of kind `mode` (pass index j of the trajectory, which sets
// the kick and drift; launch index k, which sets the field buffers) over n_tiles
// consecutive entries of `tiles`; all tiles must belong to chains of the given
// precision, dimension and tile class.  A LAST launch with j < 0 runs every
// chain's own last pass (j = n_pass - 1), with its launch index j / 2 + 1 when
// k != 0 (middle steps two per launch) or j when k == 0.
hipError_t launch_lattice_pass(int precision, int ndim, int cls, int mode, const ChainDev* chains,
                               const Tile* tiles, int n_tiles, int j, int k, hipStream_t s);

}  // namespace ihmc
