// nh_policy.cpp -- host-only part of the serving path (see nh_policy.h) and
// the C-ABI helpers nh_serve_job_team, nh_serve_job_bytes and
// nh_serve_admit_select of include/nefty_heat.h.
#include "nh_policy.h"

#include "nefty_heat.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace nhp {

namespace {
size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
}  // namespace

JobGeom job_geom(int nx, int ny, int nz, int cap) {
  JobGeom g{};
  g.TX = nx > 32 ? 64 : (nx > 16 ? 32 : 16);
  g.TY = kBlock / g.TX;
  g.txs = g.TX == 64 ? 6 : (g.TX == 32 ? 5 : 4);
  g.ntx = (nx + g.TX - 1) / g.TX;
  g.nty = (ny + g.TY - 1) / g.TY;
  const long long ng = (long long)nx * ny * nz;
  const long long xy = (long long)g.ntx * g.nty;
  const long long want = std::max<long long>(1, (ng + kVoxelsPerBlock - 1) / kVoxelsPerBlock);
  const long long want_ntz = std::max<long long>(1, (want + xy - 1) / xy);
  int tz = (int)((nz + want_ntz - 1) / want_ntz);
  if (tz < 4) tz = std::min(4, nz);
  g.TZ = tz;
  g.ntz = (nz + tz - 1) / tz;
  g.ntiles = (int)(xy * g.ntz);
  g.team = std::max(1, std::min(g.ntiles, cap));
  return g;
}

JobGeom job_geom_res(int nx, int ny, int nz) {
  JobGeom g{};
  g.TX = kResTX;
  g.TY = kResBlock / kResTX;
  g.txs = 6;
  g.ntx = (nx + g.TX - 1) / g.TX;
  g.nty = (ny + g.TY - 1) / g.TY;
  g.ntz = (nz + kResTZ - 1) / kResTZ;
  g.TZ = (nz + g.ntz - 1) / g.ntz;
  g.ntiles = (int)((long long)g.ntx * g.nty * g.ntz);
  g.team = g.ntiles;
  return g;
}

size_t job_bytes(int nx, int ny, int nz, int nsteps, int team) {
  const size_t ng = (size_t)nx * ny * nz, nxy = (size_t)nx * ny, N = (size_t)nsteps;
  size_t b = 0;
  b += align256(4 * ng) * 12;                               // alpha, z, p, u1, w0, w1, s0, s1, mu[4]
  b += align256(4 * ng * N);                                // trajectory T^1..T^N
  b += align256(8 * ng);                                    // dL/dalpha (FP64)
  b += align256(4 * nxy) + 3 * align256(4 * nxy * N);       // q_xy, target, S, dL/dS
  b += align256(4 * N);                                     // source scale per step
  b += 2 * align256(4 * 2 * N) + align256(8 * 2 * N);       // per-step iterations, status, residuals
  b += align256(kSlotBytes * (2 * (size_t)team + 2));       // team reduction slots (2 banks)
  b += align256(8 * kMseBlocks) + 256;                      // MSE partials, loss
  return b;
}

bool job_params_ok(int nx, int ny, int nz, double h, double dt, int nsteps, double rtol, int max_iter) {
  return nx >= 1 && ny >= 1 && nz >= 1 && nsteps >= 1 && dt > 0 && std::isfinite(dt) && h > 0 &&
         std::isfinite(h) && rtol > 0 && rtol < 1 && max_iter >= 1 && max_iter <= kMaxIterLimit;
}

template <typename T>
static long long first_bad_t(const T* v, size_t n, bool positive) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(v[i]) || (positive && !(v[i] > 0))) return (long long)i;
  return -1;
}
long long first_bad(const float* v, size_t n, bool positive) { return first_bad_t(v, n, positive); }
long long first_bad(const double* v, size_t n, bool positive) { return first_bad_t(v, n, positive); }

}  // namespace nhp

extern "C" {

int nh_serve_job_team(int nx, int ny, int nz, int max_blocks, int resident) {
  if (nx < 1 || ny < 1 || nz < 1 || max_blocks < 1) return 0;
  if (resident) {
    const int team = nhp::job_geom_res(nx, ny, nz).team;
    return team <= max_blocks ? team : 0;
  }
  return nhp::job_geom(nx, ny, nz, std::max(1, max_blocks / 2)).team;
}

size_t nh_serve_job_bytes(int nx, int ny, int nz, int nsteps, int team_blocks) {
  if (nx < 1 || ny < 1 || nz < 1 || nsteps < 1 || team_blocks < 1) return 0;
  return nhp::job_bytes(nx, ny, nz, nsteps, team_blocks);
}

int nh_serve_admit_select(const size_t* qbytes, const int* qteams, const double* qdur, int n_queued,
                          const size_t* abytes, const int* ateams, const double* arem, int n_active,
                          double budget_bytes, int max_blocks, int backfill, int* selected) {
  if (!qbytes || !qteams || !selected || n_queued < 1) return 0;
  if (n_active > 0 && (!abytes || !ateams || !arem)) return 0;
  if (backfill && !qdur) return 0;
  struct Act {
    double rem;
    size_t bytes;
    int team;
  };
  std::vector<Act> act;
  double used_m = 0.0;
  long long used_b = 0;
  for (int i = 0; i < n_active; ++i) {
    act.push_back({arem[i], abytes[i], ateams[i]});
    used_m += (double)abytes[i];
    used_b += ateams[i];
  }
  int n = 0;
  bool reserved = false;
  double shadow = 0.0, extra_m = 0.0;
  long long extra_b = 0;
  for (int i = 0; i < n_queued; ++i) {
    const bool fits = used_m + (double)qbytes[i] <= budget_bytes && used_b + qteams[i] <= max_blocks;
    if (!reserved) {
      if (fits) {
        used_m += (double)qbytes[i];
        used_b += qteams[i];
        act.push_back({backfill ? qdur[i] : 0.0, qbytes[i], qteams[i]});
        selected[n++] = i;
        continue;
      }
      if (!backfill) break;
      // the first job that does not fit holds a reservation: the shadow time
      // is when enough running jobs have ended for it to fit, and the extra
      // room is what it leaves free then
      reserved = true;
      std::sort(act.begin(), act.end(), [](const Act& x, const Act& y) { return x.rem < y.rem; });
      double free_m = budget_bytes - used_m;
      long long free_b = (long long)max_blocks - used_b;
      for (const Act& x : act) {
        if (free_m >= (double)qbytes[i] && free_b >= qteams[i]) break;
        free_m += (double)x.bytes;
        free_b += x.team;
        shadow = x.rem;
      }
      extra_m = free_m - (double)qbytes[i];
      extra_b = free_b - qteams[i];
      continue;
    }
    // behind the reservation: jobs that fit now and either end before the
    // shadow time or use only the extra room
    if (!fits) continue;
    const bool early = qdur[i] <= shadow;
    const bool spare = qteams[i] <= extra_b && (double)qbytes[i] <= extra_m;
    if (!early && !spare) continue;
    if (!early) {
      extra_b -= qteams[i];
      extra_m -= (double)qbytes[i];
    }
    used_m += (double)qbytes[i];
    used_b += qteams[i];
    selected[n++] = i;
  }
  return n;
}

}  // extern "C"
