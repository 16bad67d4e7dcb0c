// sph_internal.h -- device data layout shared by the HIP kernels and the host
// orchestration of the SPH library (gfx950).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sph.h"

namespace sph {

// ---------------------------------------------------------------- constants
constexpr int kWave = 64;
constexpr int kDirs = 26;        // neighbour directions {-1,0,1}^3 \ 0
constexpr int kSortDirs = 13;    // stored orderings (Sec. 3.3): half of the 26
constexpr int kSelfDir = 26;     // direction code of a self interaction
constexpr int kMaxSources = 27;  // self + 26 neighbours (single-level grid)
constexpr int kSweepWaves = 4;   // wavefronts per target cell in the interaction kernels
constexpr int kAllWaves = 4;     // wave code of a source shared by every wavefront (self)
constexpr int kMaxDepth = 12;    // levels below the top grid in the hierarchical decomposition
constexpr int kTreeSourcesPerParticle = 32;  // bound on list entries per particle (hierarchy)
constexpr double kPi = 3.14159265358979323846;

// device status bits (accumulated with atomicOr, read back by the host)
enum : uint32_t {
    ST_NONFINITE = 1u << 0,
    ST_H_TOO_LARGE = 1u << 1,
    ST_REBUILD = 1u << 2,      // some h wants to exceed what the cells allow
    ST_NOT_CONVERGED = 1u << 3,
    ST_CAPACITY = 1u << 4,
};

// ---------------------------------------------------------------- boxes
// One periodic box of the batch.  Grid dims and edges are written on the
// device (they depend on the largest h) by the grid-dims kernel.
struct BoxInfo {
    double L[3];          // box lengths
    double e_target;      // edge holding cell_target particles at mean density
    int64_t begin, n;     // particle range in caller order
    int32_t nc[3];        // cells per dimension (device-written)
    int32_t map_off;      // offset of this box's dense cell map
    int32_t map_cap;      // capacity of the dense cell map (host upper bound)
    int32_t cap_nc[3];    // per-dimension bound on nc (host)
    int32_t depth;        // levels below the top grid encoded in the keys (0: single level)
    double e[3];          // cell edges (device-written)
    double hmax;          // largest h in the box (device-written)
    double drift;         // largest displacement of a particle since the cells were built
                          // (device-written by a refresh; 0 after a build)
};

// ---------------------------------------------------------------- cells
// A cell of the decomposition: a top-grid cell, or a leaf of the hierarchy
// below it (a cube of edge e / 2^level).  Corners are integer coordinates in
// units of the finest edge e / 2^depth of the box.
struct CellInfo {
    int32_t start;        // first particle (cell order)
    int32_t count;
    int32_t box;
    int32_t c[3];         // lower corner in finest-level units
    int32_t level;        // 0: top grid
    float hlim;           // largest h the cell's interaction lists cover
};

// An interaction source of a target cell: the source cell, the direction
// along which its ordering is swept (0..25, or kSelfDir), the wavefront that
// sweeps it (kAllWaves: shared, the self source), and the position of the
// source's corner relative to the target's corner in finest-level units
// (periodic images included).
struct Source {
    int32_t cell;
    int8_t dir;
    int8_t wave;
    int16_t ox, oy, oz;
};

// Directions.  Index d in 0..25 enumerates (dx,dy,dz) in {-1,0,1}^3 \ 0 in
// lexicographic order, skipping the centre; d and 25-d are opposite.  The 13
// stored orderings are those of d = 13..25 (first non-zero component
// positive); a direction d < 13 uses stored ordering 12-d traversed in
// reverse.
__host__ __device__ inline void dir_off(int d, int o[3])
{
    int idx = d < 13 ? d : d + 1;
    o[0] = idx / 9 - 1;
    o[1] = (idx / 3) % 3 - 1;
    o[2] = idx % 3 - 1;
}
__host__ __device__ inline int dir_sort(int d) { return d < 13 ? 12 - d : d - 13; }
__host__ __device__ inline bool dir_flip(int d) { return d < 13; }
__host__ __device__ inline void dir_unit(int d, float u[3])
{
    int o[3];
    dir_off(d, o);
    int nz = (o[0] != 0) + (o[1] != 0) + (o[2] != 0);
    float s = nz == 1 ? 1.0f : (nz == 2 ? 0.70710678118654752f : 0.57735026918962576f);
    u[0] = o[0] * s; u[1] = o[1] * s; u[2] = o[2] * s;
}

// ---------------------------------------------------------------- morton
__host__ __device__ inline uint64_t spread3(uint32_t v)
{
    uint64_t x = v & 0x1fffffu;
    x = (x | x << 32) & 0x1f00000000ffffull;
    x = (x | x << 16) & 0x1f0000ff0000ffull;
    x = (x | x << 8) & 0x100f00f00f00f00full;
    x = (x | x << 4) & 0x10c30c30c30c30c3ull;
    x = (x | x << 2) & 0x1249249249249249ull;
    return x;
}

__host__ __device__ inline uint32_t compact3(uint64_t x)
{
    x &= 0x1249249249249249ull;
    x = (x ^ (x >> 2)) & 0x10c30c30c30c30c3ull;
    x = (x ^ (x >> 4)) & 0x100f00f00f00f00full;
    x = (x ^ (x >> 8)) & 0x1f0000ff0000ffull;
    x = (x ^ (x >> 16)) & 0x1f00000000ffffull;
    x = (x ^ (x >> 32)) & 0x1fffffull;
    return (uint32_t)x;
}

__host__ __device__ inline uint64_t morton3(uint32_t x, uint32_t y, uint32_t z)
{
    return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}

// ---------------------------------------------------------------- kernel parameters
// One entry of a per-cell ordering (Sec. 3.3): the projection of the particle
// on the ordering's axis when the ordering was made, and the particle's index
// within its cell.
struct SortRec {
    float key;
    uint32_t idx;
};

struct PassConsts {
    double n_ngb, tol, gamma, alpha, beps;
    int max_iter;
    double h_margin;
    double cfl;         // C_CFL of Eq. (6)
    int balsara_div;    // 1: |div v| over the Balsara denominator, 0: |curl v|
    int shared_min;     // cells of more particles than this are swept shared
    int fixed_h;        // 1: every sum at the given h, no iteration
};

}  // namespace sph
