// nh_policy.h -- host-only part of the serving path: a job's tiling, team and
// device bytes, the checks of a submitted job, and the admission order. Plain
// C++ with no HIP dependence, so that it can also be built and exercised on
// the CPU on its own (with the compiler's address and undefined-behaviour
// sanitizers).
#pragma once

#include <stddef.h>

namespace nhp {

constexpr int kBlock = 1024;                 // threads of a streaming workgroup
constexpr int kResBlock = 512;               // threads of a register-resident workgroup
constexpr int kResTX = 64;                   // resident tile: 64 x 8 columns
constexpr int kResTZ = 32;                   //   of at most 32 cells
constexpr long long kVoxelsPerBlock = 32768; // streaming tile size the planner aims at
constexpr int kMseBlocks = 64;               // workgroups of the MSE kernel (partial sums)
constexpr size_t kSlotBytes = 64;            // one team-reduction slot
constexpr int kMaxIterLimit = 30000;         // max_iter of a job (its reductions per step stay below 2^16)

// Tiling of one job: tile extents, tile counts and the team (workgroups).
struct JobGeom {
  int TX, TY, TZ, txs;
  int ntx, nty, ntz, ntiles;
  int team;
};

// Streaming tiles: x-y tiles of kBlock columns, split in z into about
// ng / kVoxelsPerBlock tiles (at least 4 planes each), one workgroup per tile
// up to `cap` workgroups.
JobGeom job_geom(int nx, int ny, int nz, int cap);

// Register-resident tiles: 64 x 8 columns and at most 32 cells in z, one
// workgroup per tile.
JobGeom job_geom_res(int nx, int ny, int nz);

// Device bytes a job holds while admitted.
size_t job_bytes(int nx, int ny, int nz, int nsteps, int team);

// The scalar parameters of a submitted job are valid.
bool job_params_ok(int nx, int ny, int nz, double h, double dt, int nsteps, double rtol, int max_iter);

// Index of the first value that is not finite (or, with positive, not > 0),
// or -1 when every value passes.
long long first_bad(const float* v, size_t n, bool positive);
long long first_bad(const double* v, size_t n, bool positive);

}  // namespace nhp
