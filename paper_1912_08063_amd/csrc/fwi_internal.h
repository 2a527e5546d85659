// fwi_internal.h -- device-side job table shared by the HIP kernels and the
// host runtime of libfwi.so (not part of the public C ABI).
//
// Field layout in HBM (one fp32 "field" = one padded grid plus a zero frame):
//   padded grid = model grid + nb sponge cells on every face (nz, ny, nx;
//   ny == 1 in 2-D), surrounded by M = order/2 ghost cells that stay zero
//   (the Dirichlet frame the star stencil reads past the sponge).
//   element (z, y, x) of the padded grid lives at
//       ((z + M) * nya + (y + gy)) * pitch + (x + M)
//   with gy = M in 3-D (0 in 2-D), nya = ny + 2 gy rows per plane and pitch a
//   multiple of 64 floats (256 B), so every row starts on a 256-byte line.
//   Tiles are aligned to memory columns [64 t, 64 t + 64), not to the grid:
//   each wavefront then loads and stores whole aligned 256-byte segments.
#pragma once
#include <stdint.h>

namespace fwi {

constexpr int kTileX = 64;   // memory columns per tile (one wavefront)
// 3-D blocks hold 4 or 8 wavefronts of 64 lanes, each thread owning 2 or 4
// consecutive y rows: a tile is 64 (x) by rows * wavefronts (y)
constexpr int kGatherThreads = 256;
// Tiling flags of 3-D step launches.  kTileZFast: the z chunk is the fastest
// index of a tile number (the chunks of one column are consecutive blocks),
// otherwise the slowest.  kTileZAlt: odd chunks march down (from their last
// plane to their first), so two neighbouring chunks read the planes around
// their common boundary at the same time, at the start or at the end of
// both, instead of once at the start and once at the end.
constexpr int32_t kTileZFast = 1;
constexpr int32_t kTileZAlt = 2;

// Size of the fixed per-GPU workspace of fwi_forward_noalloc.
constexpr uint64_t kScratchBytes = 128ull << 20;

struct Job {
    // geometry of the padded grid and its field layout
    int32_t nz, ny, nx;    // padded grid (ny == 1 in 2-D)
    int32_t pitch;         // floats per row
    int32_t nya;           // rows per plane, ghost rows included
    int32_t nb;            // sponge width
    int64_t plane;         // floats per plane (nya * pitch)
    int64_t fstride;       // floats per field allocation
    float eta_dt;          // eta_max * dt / nb^2: eta*dt = eta_dt * sum_a d_a^2
    float src_scale;       // dt^2 / dx^D
    // tiling of the step kernels: tile[0] forward launches, tile[1] adjoint
    // launches (their blocks may differ in shape)
    struct Tiling {
        int32_t ntx, nty, nzc, zc;   // tiles in x and y, z chunks and chunk length
        int32_t ntiles;              // ntx * nty * nzc
        int32_t flags;               // kTile* bits (3-D launches only)
    } tile[2];
    int32_t ngather;             // gather blocks (forward record)
    // time: forward n = n0 + step, adjoint k = k0 - step; a launch updates a
    // job only for n in [fwd_lo, fwd_hi) (forward) or k in [adj_lo, adj_hi)
    int32_t n0;
    int32_t k0;
    int32_t fwd_lo, fwd_hi;
    int32_t adj_lo, adj_hi;
    int32_t nt;
    int32_t record;        // forward: write traces
    int32_t accumulate;    // adjoint: accumulate the gradient
    // fields
    const float *kappa;    // (v dt / dx)^2 on the padded grid (frame = 0)
    float *ring;           // forward wavefield ring, level n in slot n mod R
    int32_t R;
    float *adj;            // adjoint ring, level k in slot k mod 2
    float *grad;           // sum_n psi^{n+1} * lap'(p^n)
    float *snap;           // snapshot store, slot s holds 2 fields
    // point source (padded coordinates, -1: none)
    int32_t src_z, src_y, src_x;
    int32_t nrec;
    const float *wavelet;  // [nt]
    const int64_t *rec_off;    // [nrec] field offsets of the receiver cells
    const int32_t *rec_next;   // [nrec] next receiver on the same cell, -1 at the end
    const int32_t *rec_head;   // [nrec] 1 for the first receiver of its cell
    // 2-D adjoint source: the first receiver of each receiver cell, grouped
    // by the adjoint tile that holds the cell and sorted by row within it;
    // tile t (local index) owns entries rt_start[t] .. rt_start[t+1]-1 of
    // rt_rec (receiver) and rt_key (row << 6 | column within the tile)
    const int32_t *rt_start;   // [adjoint tiles + 1] (2-D jobs only)
    const int32_t *rt_rec;     // [receiver cells]
    const int32_t *rt_key;     // [receiver cells]
    float *traces;         // [nt][nrec]
    const float *res;      // [nt][nrec] adjoint source
    // per-round time levels of a serving chunk (nullptr: n0 + step / k0 - step)
    const int32_t *lev;
};

// Forward levels that a launch finds in the snapshot store instead of the
// ring: level lev[i] is field fld[i] of each job's store (slot s holds fields
// 2s and 2s+1).  Binomial checkpointing uses it to read a restored state, or
// write a state it is about to snapshot, in place instead of copying it.
// Unused entries hold kNoLevel.
constexpr int32_t kNoLevel = -2147483647 - 1;
struct LevelMap {
    int32_t lev[3] = {kNoLevel, kNoLevel, kNoLevel};
    int32_t fld[3] = {0, 0, 0};
};

// Launch tables of fwi_jobs_advance, assembled on the device (k_assemble):
// each entry is copied from the job's own table entry in its memory and its
// time window for this chunk is patched in.  Passed by value as a kernel
// argument, so the host neither copies tables nor waits for the stream.
constexpr int kAssembleJobs = 16;
constexpr int kAssemblePrefix = 64;
constexpr int kAssembleLevels = 384;
struct AssembleArgs {
    int32_t count;                  // entries first .. first + count - 1
    int32_t first;
    int32_t nprefix;                // prefix ints pfirst .. pfirst + nprefix - 1
    int32_t pfirst;
    int32_t nlev;                   // level-list ints lfirst .. lfirst + nlev - 1
    int32_t lfirst;
    const Job *src[kAssembleJobs];  // the job's own table entry (device)
    int32_t win[kAssembleJobs][7];  // n0, k0, fwd_lo, fwd_hi, adj_lo, adj_hi, record
    int32_t levoff[kAssembleJobs];  // entry's level list in the group's lists (-1: none)
    int32_t prefix[kAssemblePrefix];
    int32_t lev[kAssembleLevels];
};
static_assert(sizeof(AssembleArgs) <= 4000, "kernel arguments are limited to 4 KB");

}  // namespace fwi
