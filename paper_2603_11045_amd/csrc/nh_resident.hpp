// nh_resident.hpp -- register-resident variant of the per-step kernel (FP32).
//
// When every tile of the grid fits one workgroup per CU (a tile is 512
// columns of at most kResTZ cells), the CG state of a tile -- p, u = r/D,
// A u / D and A p / D, the vectors of the single-reduction iteration of
// nh_kernels.hpp -- stays in the registers of the workgroup that owns the tile
// for the whole time step, and 1/alpha stays in LDS. Only x, which no neighbour
// reads during the solve, is updated in place in memory inside each
// iteration's sweep (8 bytes per cell and iteration, coalesced, no halo). The
// elementwise updates run in registers, the stencil exchanges in-tile
// neighbours through LDS a few z-planes per workgroup barrier, and only the
// values on the tile's faces are published (write-through, device-scope
// stores) for the neighbouring tiles, in the single-problem kernel the x-edge
// columns as compact copies. A neighbour loads them straight into its LDS halo
// rings (device-coherent direct loads) as soon as the team reduction that
// follows shows their slots tagged, while it still gathers the other slots.
// Because every inter-workgroup exchange uses device-coherent accesses, the
// team reduction needs no L2 write-back or invalidation. The arithmetic is the
// same as the streaming kernel's single-reduction form; halo values are
// recomputed with the same fused multiply-adds as the owner uses, so both
// sides see identical bits.
#pragma once

#include "nh_kernels.hpp"

namespace nh {

constexpr int kResBlock = 512;              // one workgroup (8 wave64, 256 VGPRs each) per CU
constexpr int kResTZ = 32;                  // max cells per column of a tile
constexpr int kRing = 144;                  // max 2*(TX+TY) with TX*TY = 512
constexpr int kResPlane = 660;              // max (TX+2)*(TY+2) with TX*TY = 512

__device__ __forceinline__ void st_dev(float* p, float v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float ld_dev(const float* p) {
  return __hip_atomic_load(const_cast<float*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
constexpr int kCpolSc1 = 16;                // cache policy of a device-coherent load (sc1), as ld_dev

// Buffer access to one FP32 vector of n elements: a lane's element offset
// (bytes, per lane) plus a plane offset (bytes, uniform) -- no per-lane 64-bit
// address arithmetic. A lane whose offset is kNoLane reads 0 and writes
// nothing (out of the buffer's range), which replaces a lane condition.
constexpr unsigned kNoLane = 0x80000000u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t vec_rsrc(const float* p, long long n) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(p), 0, (int)(n * 4), 0x00020000);
}
template <int CPOL = 0>
__device__ __forceinline__ float buf_ld(__amdgpu_buffer_rsrc_t r, unsigned voff, int soff) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, CPOL));
}
template <int CPOL = 0>
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, unsigned voff, int soff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, CPOL);
}

struct ResRed {
  double red[2][kMaxWaves][kNumRed];        // two buffers of per-wave partials (block_sum)
  double bc[kNumRed];
  int flag;
};

// LDS layout of the resident kernel (bytes).
constexpr size_t kResAlphaFloats = (size_t)(kResTZ + 2) * kResPlane;   // alpha tile + halos
constexpr int kResPZ = 3;                   // planes per barrier in one-vector sweeps
constexpr size_t kResPlaneFloats = 2 * (size_t)kResPZ * kResPlane;     // [2 sets][kResPZ] or [2 vectors][2]
constexpr size_t kResRingFloats = 3 * (size_t)kResTZ * kRing;          // [3 vectors][TZ][ring]
constexpr size_t kResLdsBytes =
    (kResAlphaFloats + kResPlaneFloats + kResRingFloats) * sizeof(float) + sizeof(ResRed) + 64;

// Team reduction of the resident and blocked kernels. Every workgroup stores
// its sum in its own slot, then EVERY workgroup gathers all slots and sums them
// in the same fixed order, so all obtain bit-identical results after one
// exchange (no master round trip). Each FP64 value travels as two 64-bit words
// (tag << 32 | one half of its bits), the tag being the low 32 bits of the
// reduction's epoch: a reader takes a slot's values and their validity in one
// load round trip, and the writer issues its words without waiting between
// them. Tags are unique between clears of the slots: an epoch is
// (launch << 24) + k with k < 2^24 reductions per launch, and the host zeroes
// the slots every 256 launches (tag 0 is never used) and whenever the slots
// held the untagged layout of team_sum. Slots alternate between two banks by
// epoch parity: a workgroup can be at most one reduction ahead of the slowest
// reader (the next reduction needs every workgroup's slot), so a bank is
// never rewritten while still read. Every value another workgroup reads was
// written with device-scope stores, and every wave waits for its own stores
// before the workgroup's block sum, so the tags are issued after the
// workgroup's earlier stores have completed: the reduction doubles as the
// team's barrier with no cache maintenance. Slots: 2 * team.
struct alignas(64) TSlot {
  unsigned long long w[2 * kNumRed];
};
static_assert(sizeof(TSlot) == sizeof(Slot), "the slot buffers are sized for either layout");

__device__ __forceinline__ void st_tag(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// No work to start once the neighbours have published (see team_sum_dev).
struct NoNeighbours {
  __device__ int rank(int) const { return -1; }
  __device__ void ready() const {}
};

// nbr.rank(k), k < 6, gives the ranks of the workgroups whose tiles share a
// face with this one (-1: none); once every one of them has published its slot
// for this reduction -- so their earlier stores are visible -- every wave calls
// nbr.ready(), which may start loads of what the neighbours published, before
// it gathers slots. (Keeping those loads to the waves that gather no slots
// measured slower.)
template <int NV, int BLOCK = kResBlock, class Nbr = NoNeighbours>
__device__ __forceinline__ bool team_sum_dev(const StepArgs<float>& S, int rank, unsigned long long& epoch,
                                             double (&v)[NV], ResRed* rs, const Nbr& nbr = Nbr()) {
  static_assert(NV <= kNumRed, "slot too small");
  __builtin_amdgcn_s_waitcnt(0);
  block_sum<NV, BLOCK / 64>(v, rs->red[0]);
  if (S.team == 1) {
    __syncthreads();                        // red[0] is free again
    return true;
  }
  const unsigned long long e = ++epoch;
  const unsigned tag = (unsigned)e;
  const unsigned long long th = (unsigned long long)tag << 32;
  TSlot* slots = (TSlot*)S.slots + (size_t)(e & 1) * S.team;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const unsigned long long bits = (unsigned long long)__double_as_longlong(v[i]);
      st_tag(&slots[rank].w[2 * i], th | (bits & 0xffffffffull));
      st_tag(&slots[rank].w[2 * i + 1], th | (bits >> 32));
    }
  }
  int ok = 1;
  {
    // every wave waits (lanes 0-5) for the neighbours' slots, then starts its loads
    const int k = threadIdx.x & 63;
    const int b = k < 6 ? nbr.rank(k) : -1;
    if (b >= 0 && b != rank) {
      const long long t0 = wall_clock64();
      while (true) {
        bool all = true;
#pragma unroll
        for (int j = 0; j < 2 * NV; ++j) all &= (unsigned)(ld_epoch(&slots[b].w[j]) >> 32) == tag;
        if (all) break;
        __builtin_amdgcn_s_sleep(1);
        if (wall_clock64() - t0 > S.timeout_ticks) { ok = 0; break; }
      }
    }
    nbr.ready();
  }
  double s[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) s[i] = 0.0;
  for (int b = threadIdx.x; b < S.team; b += BLOCK) {
    if (b == rank) {
#pragma unroll
      for (int i = 0; i < NV; ++i) s[i] += v[i];
      continue;
    }
    unsigned long long w[2 * NV];
    const long long t0 = wall_clock64();
    while (true) {
      bool all = true;
#pragma unroll
      for (int k = 0; k < 2 * NV; ++k) {
        w[k] = ld_epoch(&slots[b].w[k]);
        all &= (unsigned)(w[k] >> 32) == tag;
      }
      if (all) break;
      __builtin_amdgcn_s_sleep(1);
      if (wall_clock64() - t0 > S.timeout_ticks) { ok = 0; break; }
    }
#pragma unroll
    for (int i = 0; i < NV; ++i)
      s[i] += __longlong_as_double((long long)((w[2 * i + 1] << 32) | (w[2 * i] & 0xffffffffull)));
  }
  ok = __syncthreads_and(ok);
  block_sum<NV, BLOCK / 64>(s, rs->red[1]);
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = s[i];
  if (!ok && threadIdx.x == 0) atomicOr(S.err_flag, (int)kTimeout);
  return ok != 0;
}

// Compile-time tile geometry: TX columns in x (a power of two), 512 / TX in y.
template <int TX_>
struct RG {
  static constexpr int TX = TX_;
  static constexpr int TY = kResBlock / TX_;
  static constexpr int PW = TX + 2;
  static constexpr int PL = (TX + 2) * (TY + 2);
  static constexpr int RING = 2 * (TX + TY);
  static_assert(PL <= kResPlane && RING <= kRing, "tile too large");
};

// LDS layout of a ring buffer (the values of one vector on the tile's halo
// ring, every plane of the tile), side by side so that a wave's direct load
// of 64 consecutive slots is one halo row of one plane (the -y and +y sides,
// 64 cells each) or the 8 halo cells of the -x or +x side on 8 consecutive
// planes: [-y: TZ][64] [+y: TZ][64] [-x: TZ][8] [+x: TZ][8].
constexpr int kRingRowN = kResTZ * 64;                     // one row side
constexpr int kRingColN = kResTZ * 8;                      // one column side
constexpr int kRingYm = 0, kRingYp = kRingRowN, kRingXm = 2 * kRingRowN, kRingXp = 2 * kRingRowN + kRingColN;
static_assert(2 * kRingRowN + 2 * kRingColN == kResTZ * kRing, "ring layout");

// Ring cell h in the order of ring_cell (h < TX: -y row, then +y row, -x
// column, +x column) at plane z: its slot in a ring buffer is base + z * stride.
__device__ __forceinline__ void ring_slot(int h, int& base, int& stride) {
  if (h < 64) { base = kRingYm + h; stride = 64; }
  else if (h < 128) { base = kRingYp + h - 64; stride = 64; }
  else if (h < 136) { base = kRingXm + h - 128; stride = 8; }
  else { base = kRingXp + h - 136; stride = 8; }
}

// Where one thread of the resident workgroup sits in its tile.
struct ResPos {
  int tid;                                  // thread index (laundered by the caller)
  int tx, ty;
  int x0, y0, z0, tzn;
  int gx, gy;
  bool own;
  int col;                                  // x + nx*y (the grid has fewer than 2^31 cells)
  int oslot;
  bool top_z, bot_z;                        // a tile exists below (z0-1) / above (z1)
  bool edge;                                // column on the tile's x/y boundary
  bool yedge;                               // with compact x-edge columns: column on the y boundary
  int xside;                                //   and 0 first, 1 last column in x, else -1
};

// Geometry of ring cell h (0 <= h < RING): grid column and LDS plane slot.
template <class G>
__device__ __forceinline__ void ring_cell(const Geom& g, const ResPos& q, int h, bool& in, int& hcol,
                                          int& hslot) {
  int hx, hy;
  constexpr int TX = G::TX, TY = G::TY, PW = G::PW;
  if (h < TX) { hx = q.x0 + h; hy = q.y0 - 1; hslot = h + 1; }
  else if ((h -= TX) < TX) { hx = q.x0 + h; hy = q.y0 + TY; hslot = (TY + 1) * PW + h + 1; }
  else if ((h -= TX) < TY) { hx = q.x0 - 1; hy = q.y0 + h; hslot = (h + 1) * PW; }
  else { h -= TY; hx = q.x0 + TX; hy = q.y0 + h; hslot = (h + 1) * PW + TX + 1; }
  in = hx >= 0 && hx < g.nx && hy >= 0 && hy < g.ny;
  hcol = in ? hx + g.nx * hy : 0;
}

// Fill an LDS ring buffer for every plane of the tile: ring[slot(z, h)] =
// val(global index) for in-grid ring cells, 0 outside. All loads of a thread
// are issued before the first LDS store, so the fill costs one memory latency.
template <class G, typename F>
__device__ __forceinline__ void fill_ring(const Geom& g, const ResPos& q, float* ring, F val) {
  static_assert(G::TX == 64 && G::TY == 8, "ring layout assumes 64 x 8 tiles");
  constexpr int kMaxPer = (G::RING * kResTZ + kResBlock - 1) / kResBlock;
  const int n = G::RING * q.tzn;
  float v[kMaxPer];
  int slot[kMaxPer];
#pragma unroll
  for (int k = 0; k < kMaxPer; ++k) {
    const int e = q.tid + k * kResBlock;
    v[k] = 0.f;
    slot[k] = -1;
    if (e < n) {
      const int z = e / G::RING, h = e - z * G::RING;
      bool in;
      int hcol, hslot, base, stride;
      ring_cell<G>(g, q, h, in, hcol, hslot);
      ring_slot(h, base, stride);
      slot[k] = base + z * stride;
      if (in) v[k] = val(hcol + (q.z0 + z) * (int)g.nxy);
    }
  }
#pragma unroll
  for (int k = 0; k < kMaxPer; ++k)
    if (slot[k] >= 0) ring[slot[k]] = v[k];
}

// Face weights and the diagonal of one cell, from the 1/alpha tile in LDS
// (lz = z + 1 is the cell's plane).
struct Nb {
  float w[6];                               // -x +x -y +y -z +z
  float D;
};

template <class G>
__device__ __forceinline__ Nb faces_at(const float* la, const ResPos& q, int z, float sx, float sy, float sz) {
  const float* pl = la + (z + 1) * G::PL + q.oslot;
  const float ia = pl[0];
  Nb n;
  n.w[0] = face_w<float>(ia, pl[-1]);
  n.w[1] = face_w<float>(ia, pl[1]);
  n.w[2] = face_w<float>(ia, pl[-G::PW]);
  n.w[3] = face_w<float>(ia, pl[G::PW]);
  n.w[4] = face_w<float>(ia, pl[-G::PL]);
  n.w[5] = face_w<float>(ia, pl[G::PL]);
  n.D = diag_w<float>(sx, sy, sz, n.w);
  return n;
}

// A v at one cell given the four in-plane neighbours from LDS and the two z neighbours.
__device__ __forceinline__ float apply_at(const Nb& n, float sx, float sy, float sz, float v, const float* pl,
                                          int oslot, int PW, float vzm, float vzp) {
  const float nb[6] = {pl[oslot - 1], pl[oslot + 1], pl[oslot - PW], pl[oslot + PW], vzm, vzp};
  return apply_w<float>(sx, sy, sz, n.w, v, nb);
}

// Plane-by-plane sweep over the tile for NV staged vectors. own(k, z) gives
// the thread's own value of vector k at plane z, ring[k] the LDS ring buffers,
// zlo/zhi the values below and above the tile; cell(z, plane pointers) does the work.
// A one-vector sweep stages PZ1 (<= kResPZ) planes per barrier (groups
// alternate between two sets of plane buffers, so one barrier per group
// suffices: a set is written again two groups later, after the next group's
// barrier).
template <class G, int NV, int PZ1, typename OwnF, typename RingF, typename CellF>
__device__ __forceinline__ void plane_sweep_r(const Geom& g, const ResPos& q, float* lp, RingF ringv,
                                              OwnF own, const float (&zlo)[2], const float (&zhi)[2], CellF cell) {
  static_assert(PZ1 >= 1 && PZ1 <= kResPZ, "plane buffers");
  constexpr int PZ = NV == 1 ? PZ1 : 1;     // planes per barrier
  // ring cells handled by this thread for the plane copy
  // the ring cell this thread copies into the plane: its LDS plane slot, ring
  // slot base and the log2 of the ring slot stride per plane, packed in one
  // register (hslot < 1024, base < 8192)
  const int h = q.tid;
  int hpack = -1;
  if (h < G::RING) {
    bool hin;
    int hcol, hslot, rbase, rstride;
    ring_cell<G>(g, q, h, hin, hcol, hslot);
    ring_slot(h, rbase, rstride);
    hpack = hslot | (rbase << 10) | ((rstride == 64 ? 6 : 3) << 23);
  }
#pragma unroll
  for (int zg = 0; zg < kResTZ; zg += PZ) {
    if (zg < q.tzn) {
      float* pl[PZ][NV];
#pragma unroll
      for (int j = 0; j < PZ; ++j)
#pragma unroll
        for (int k = 0; k < NV; ++k)
          pl[j][k] = lp + (size_t)(PZ > 1 ? PZ * ((zg / PZ) & 1) + j : 2 * k + (zg & 1)) * kResPlane;
#pragma unroll
      for (int j = 0; j < PZ; ++j) {
        const int z = zg + j;
        if (z < kResTZ && (j == 0 || z < q.tzn)) {
#pragma unroll
          for (int k = 0; k < NV; ++k) {
            pl[j][k][q.oslot] = q.own ? own(k, z) : 0.f;
            // (laundered per plane, so that the 32 planes' ring slots are not all
            // precomputed into registers)
            int hp = hpack;
            asm volatile("" : "+v"(hp));
            if (hp >= 0) pl[j][k][hp & 1023] = ringv(k, ((hp >> 10) & 8191) + (z << (hp >> 23)));
          }
        }
      }
      __syncthreads();
      if (q.own) {
#pragma unroll
        for (int j = 0; j < PZ; ++j) {
          const int z = zg + j;
          if (z < kResTZ && (j == 0 || z < q.tzn)) {
            float vzm[NV], vzp[NV];
#pragma unroll
            for (int k = 0; k < NV; ++k) {
              vzm[k] = z == 0 ? zlo[k] : own(k, z > 0 ? z - 1 : 0);
              vzp[k] = z + 1 == q.tzn ? zhi[k] : own(k, z + 1 < kResTZ ? z + 1 : kResTZ - 1);
            }
            cell(z, pl[j], vzm, vzp);
          }
        }
      }
    }
  }
  __syncthreads();
}

// Plane sweep whose halo ring values are stored in LDS (NV ring buffers).
template <class G, int NV, int PZ1, typename OwnF, typename CellF>
__device__ __forceinline__ void plane_sweep(const Geom& g, const ResPos& q, float* lp, const float* ring,
                                            OwnF own, const float (&zlo)[2], const float (&zhi)[2], CellF cell) {
  plane_sweep_r<G, NV, PZ1>(g, q, lp, [&](int k, int o) { return ring[(size_t)k * kResTZ * kRing + o]; }, own,
                            zlo, zhi, cell);
}

// Rank of the workgroup owning face neighbour k (-x, +x, -y, +y, -z, +z) of
// tile `tile`, or -1 at the grid's edge (first_tile inverted).
__device__ __forceinline__ int neighbour_rank(const Geom& g, int tile, int team, int xcd, int k) {
  const int itz = tile % g.ntz, rest = tile / g.ntz;
  const int itx = rest % g.ntx, ity = rest / g.ntx;
  int t = -1;
  switch (k) {
    case 0: t = itx > 0 ? tile - g.ntz : -1; break;
    case 1: t = itx + 1 < g.ntx ? tile + g.ntz : -1; break;
    case 2: t = ity > 0 ? tile - g.ntz * g.ntx : -1; break;
    case 3: t = ity + 1 < g.nty ? tile + g.ntz * g.ntx : -1; break;
    case 4: t = itz > 0 ? tile - 1 : -1; break;
    default: t = itz + 1 < g.ntz ? tile + 1 : -1; break;
  }
  if (t < 0) return -1;
  if (xcd && (team & 7) == 0) {             // the inverse of first_tile's XCD order
    const int per = team >> 3;
    return (t % per) * 8 + t / per;
  }
  return t;
}

// The tagged reduction's early hook of the resident step: the neighbours'
// ranks and `ready`, which the reduction calls in every wave once they have
// all published.
template <typename F>
struct ResNeighbours {
  const Geom& g;
  int tile, team, xcd;
  F ready_f;
  __device__ int rank(int k) const { return neighbour_rank(g, tile, team, xcd, k); }
  __device__ void ready() const { ready_f(); }
};
template <typename F>
__device__ __forceinline__ ResNeighbours<F> res_neighbours(const Geom& g, int tile, int team, int xcd, F f) {
  return ResNeighbours<F>{g, tile, team, xcd, f};
}

// Compact copies of the tiles' x-edge columns, which the x neighbours load
// into their halo rings: [bank][tile][side][vector][kResTZ][8] floats, side 0
// the tile's first column in x, 1 its last, vectors u, w/D, s/D. Eight planes
// of one column are 64 consecutive floats, one load of a wave (in the vectors
// themselves consecutive values of a column lie nx floats apart, a cache line
// each); the offsets of a tile's vectors and planes are constants.
constexpr int kXfCol = kResTZ * 8;          // floats of one column
constexpr int kXfTile = 2 * 3 * kXfCol;     // floats per tile and bank
// column (tile 0, side 0) of vector vec in bank `bank`
__device__ __forceinline__ float* xface_of(float* xf, int team, int vec, int bank) {
  return xf + (size_t)bank * team * kXfTile + (size_t)vec * kXfCol;
}

// Start copying src's values at the tile's ring cells into an LDS ring buffer
// with direct global-to-LDS loads (device-coherent), without waiting. Each
// wave issues nine loads of 64 lanes: the -y and +y halo rows of planes w,
// w + 8, w + 16, w + 24 (lane = x offset; coalesced) and one block of eight
// planes of the -x (waves 0-3) or +x (waves 4-7) halo column (lane = 8 z + y),
// landing in 64 consecutive slots of the side-by-side layout. Lanes on cells
// outside the grid or below the tile's last plane load nothing: their slots
// must hold zeros already. (Loading the rows 16 bytes per lane, four planes
// per load, measured slower.) With xsrc the column blocks come from the
// compact copies of the x neighbours' edge columns.
template <class G>
__device__ __forceinline__ void ring_dma(const Geom& g, const ResPos& q, float* ring, const float* src, int tid,
                                         int nxy, const float* xsrc = nullptr, int tile = 0) {
  static_assert(G::TX == 64 && G::TY == 8 && kResBlock == 512, "ring loads assume 64 x 8 tiles, 8 waves");
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  // rows: x = x0 + lane at y0 - 1 and y0 + 8
  const int gx = q.x0 + lane;
  const bool row_x = gx < g.nx;
  const bool ym = row_x && q.y0 > 0, yp = row_x && q.y0 + G::TY < g.ny;
  const float* bz = src + (long long)q.z0 * nxy;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int z = wave + 8 * j;
    if (z < q.tzn) {
      const float* pz = bz + (long long)z * nxy;
      if (ym) __builtin_amdgcn_global_load_lds(pz + (gx + g.nx * (q.y0 - 1)), ring + kRingYm + 64 * z, 4, 0, kCpolSc1);
      if (yp) __builtin_amdgcn_global_load_lds(pz + (gx + g.nx * (q.y0 + G::TY)), ring + kRingYp + 64 * z, 4, 0,
                                               kCpolSc1);
    }
  }
  // columns: eight planes 8 b .. 8 b + 7 of side x0 - 1 (b = wave) or x0 + 64 (b = wave - 4)
  const int b = wave & 3;
  const bool xp = wave >= 4;
  const int cx = xp ? q.x0 + G::TX : q.x0 - 1;
  const int cz = 8 * b + (lane >> 3), cy = q.y0 + (lane & 7);
  if (cz < q.tzn && cx >= 0 && cx < g.nx && cy < g.ny) {
    // from the compact copy: the neighbour's facing column (its first for +x,
    // its last for -x), planes 8 b .. 8 b + 7, 64 consecutive floats
    const float* s = xsrc ? xsrc + (size_t)(2 * (xp ? tile + g.ntz : tile - g.ntz) + (xp ? 0 : 1)) * (3 * kXfCol) +
                                64 * b + lane
                          : bz + ((long long)cz * nxy + cx + (long long)g.nx * cy);
    __builtin_amdgcn_global_load_lds(s, ring + (xp ? kRingXp : kRingXm) + 64 * b, 4, 0, kCpolSc1);
  }
}

// One implicit-Euler step of one team with the tile's CG state in registers
// (dsm: the dynamic LDS of kResLdsBytes). Per-step fields come from V.
// publish: end with a fenced team barrier, for callers that run further steps
// in the same launch. PZ: planes per barrier of the one-vector sweeps; XF: the
// x-edge columns also go to the compact copies in S.xface (2 * team * kXfTile
// floats), from which the x neighbours load them (and not from the vectors).
template <int TXC, int PZ = kResPZ, bool XF = false>
__device__ __forceinline__ StepResult resident_step(const StepArgs<float>& S, const StepVar<float>& V, int rank,
                                                    unsigned char* dsm, bool publish) {
  using G = RG<TXC>;
  constexpr int TZ = kResTZ;
  float* la = (float*)dsm;
  float* lp = la + kResAlphaFloats;
  float* lring = lp + kResPlaneFloats;
  ResRed* rs = (ResRed*)(lring + kResRingFloats);

  const Geom& g = S.g;
  // a caller that loops over steps must not keep the tile geometry of one
  // step live into the next: the laundered indices make it per-step values
  int rank_l = rank, tid0 = threadIdx.x;
  asm volatile("" : "+s"(rank_l));
  asm volatile("" : "+v"(tid0));
  const int tile = first_tile(rank_l, S.team, S.xcd_order);
  const Tile T = tile_of(g, tile);

  ResPos q;
  q.tid = tid0;
  q.tx = tid0 % G::TX;
  q.ty = tid0 / G::TX;
  q.x0 = T.x0; q.y0 = T.y0; q.z0 = T.z0;
  q.tzn = T.z1 - T.z0;
  q.gx = T.x0 + q.tx;
  q.gy = T.y0 + q.ty;
  q.own = q.gx < g.nx && q.gy < g.ny;
  q.col = q.own ? q.gx + g.nx * q.gy : 0;
  q.oslot = (q.ty + 1) * G::PW + q.tx + 1;
  q.bot_z = T.z0 > 0;
  q.top_z = T.z1 < g.nz;
  q.edge = q.tx == 0 || q.tx == G::TX - 1 || q.ty == 0 || q.ty == G::TY - 1;
  q.yedge = XF && (q.ty == 0 || q.ty == G::TY - 1);
  q.xside = !XF ? -1 : (q.tx == 0 ? 0 : (q.tx == G::TX - 1 ? 1 : -1));
  const float sx = S.sx, sy = S.sy, sz = S.sz;
  const int nxy = (int)g.nxy;

  unsigned long long red = V.epoch_base;
  bool ok = true;
  // phase stamps (NH_TRACE_STEP) only in the traced instance: the untraced
  // one keeps no trace state live through the step
  int ntr = 0;
  const bool tr = S.trace && (rank == S.trace_rank || S.trace_rank < 0) && threadIdx.x == 0;
  long long* trace = S.trace ? S.trace + (S.trace_rank < 0 ? (long long)rank * S.trace_cap : 0) : nullptr;
  auto stamp = [&]() {
    if (tr && ntr < S.trace_cap) trace[ntr++] = wall_clock64();
  };
  stamp();

  // alpha tile with halos: planes z0-1 .. z0+tzn, each (TX+2) x (TY+2),
  // streamed straight into LDS (slot e of the tile <- lane e % 64 of a wave's
  // load); cells outside the grid are stored as zero. Once loaded, each
  // thread replaces its slots by 1/alpha (+inf outside the grid).
  const int na = (q.tzn + 2) * G::PL;
  for (int e0 = 0; e0 < na; e0 += kResBlock) {
    const int e = e0 + tid0;
    if (e < na) {
      const int lz = e / G::PL, rem = e - lz * G::PL;
      const int ly = rem / G::PW, lx = rem - ly * G::PW;
      const int gz = T.z0 - 1 + lz, gxx = T.x0 - 1 + lx, gyy = T.y0 - 1 + ly;
      if (gz >= 0 && gz < g.nz && gxx >= 0 && gxx < g.nx && gyy >= 0 && gyy < g.ny)
        __builtin_amdgcn_global_load_lds(S.alpha + gxx + g.nx * gyy + gz * nxy, la + e0 + (tid0 & ~63), 4, 0, 0);
      else
        la[e] = 0.f;
    }
  }

  // rings 1 and 2 receive only in-grid values by direct loads: their other
  // slots stay zero (ring 0 is fully rewritten by the set-up's fill)
  for (int e = tid0; e < 2 * kResTZ * kRing; e += kResBlock) lring[kResTZ * kRing + e] = 0.f;

  float pr[TZ], ur[TZ], wr[TZ], sr[TZ];
#pragma unroll
  for (int z = 0; z < TZ; ++z) { pr[z] = 0.f; ur[z] = 0.f; wr[z] = 0.f; sr[z] = 0.f; }
  float (&xr)[TZ] = pr;                     // x0 lives in the p registers during the set-up

  // ---------------- set-up: x0, b, r = b - A x0, u = r / D; x = x0 in memory
  // x0 = h1 (the previous state), or its extrapolation e1 h1 + (e2 h2 + h3)
  const float* x0src = V.xprev;
  const int order = guess_order(V);
  const float* h2 = order >= 1 ? V.xprev2 : nullptr;
  const float* h3 = order == 2 ? V.xprev3 : nullptr;
  float e1, e2;
  guess_coef<float>(order, e1, e2);
  auto x0_of = [&](float h1v, float h2v, float h3v) -> float {
    if (!h2) return h1v;
    float v = mul_rn(e2, h2v);
    if (h3) v = add_rn(v, h3v);
    return fmaf(e1, h1v, v);
  };
  auto x0_at = [&](int i) -> float { return x0_of(x0src[i], h2 ? h2[i] : 0.f, h3 ? h3[i] : 0.f); };
  // the column's h1, h2, h3 are all loaded before any is used (h1 in the w
  // registers, h2 in the p registers, h3 in the u registers: all free until
  // the set-up sweep); h1 stays for the right-hand side, so the set-up sweep
  // waits for no load
  float (&br)[TZ] = wr;
  if (q.own && x0src) {
#pragma unroll
    for (int z = 0; z < TZ; ++z)
      if (z < q.tzn) {
        const int i = q.col + (T.z0 + z) * nxy;
        br[z] = x0src[i];
        if (h2) xr[z] = h2[i];
        if (h3) ur[z] = h3[i];
      }
#pragma unroll
    for (int z = 0; z < TZ; ++z)
      if (z < q.tzn) xr[z] = x0_of(br[z], xr[z], ur[z]);
  }
  if (q.own && x0src != V.x) {
#pragma unroll
    for (int z = 0; z < TZ; ++z)
      if (z < q.tzn) V.x[q.col + (T.z0 + z) * nxy] = xr[z];
  }
  float xtop = xr[0];                       // the latest x of the column's first cell (surface frame)
  float zlo[2] = {0.f, 0.f}, zhi[2] = {0.f, 0.f};
  if (x0src) {
    if (q.own && q.bot_z) zlo[0] = x0_at(q.col + (T.z0 - 1) * nxy);
    if (q.own && q.top_z) zhi[0] = x0_at(q.col + T.z1 * nxy);
    fill_ring<G>(g, q, lring, [&](int i) { return x0_at(i); });
  } else {
    fill_ring<G>(g, q, lring, [&](int) { return 0.f; });
  }
  // the top source, loaded before the sweep as well
  const float top_q = q.own && T.z0 == 0 ? V.top_src[q.col] : 0.f;
  __builtin_amdgcn_s_waitcnt(0);            // the alpha tile has reached LDS
  // (a wave's direct loads fill the slots of its own threads)
  for (int e = tid0; e < na; e += kResBlock) la[e] = inv_alpha<float>(la[e]);
  __syncthreads();
  double acc3[3] = {0.0, 0.0, 0.0};
  plane_sweep<G, 1, PZ>(g, q, lp, lring, [&](int, int z) { return xr[z]; }, zlo, zhi,
                 [&](int z, float* const* pl, const float* vzm, const float* vzp) {
                   const Nb n = faces_at<G>(la, q, z, sx, sy, sz);
                   const float Av = apply_at(n, sx, sy, sz, xr[z], pl[0], q.oslot, G::PW, vzm[0], vzp[0]);
                   float b = h2 ? br[z] : xr[z];
                   if (T.z0 + z == 0) b += V.top_scale * top_q;
                   const float r = b - Av;
                   const float u = r * rcp<float>(n.D);
                   ur[z] = u;
                   const double bd = b, rd = r;
                   acc3[0] += bd * bd;
                   acc3[1] += rd * (double)u;
                   acc3[2] += rd * rd;
                 });
  stamp();
  // publish u0 on the tile's faces (x-edge columns: the compact copy)
  float* const xf = XF ? S.xface : nullptr;
  const bool fedge = XF ? q.yedge : q.edge;   // face cells stored in the vectors
  const int xfo = (2 * tile + q.xside) * (3 * kXfCol) + q.ty;   // the column's row, bank 0 vector 0
  if (q.own) {
#pragma unroll
    for (int z = 0; z < TZ; ++z)
      if (z < q.tzn) {
        if (fedge || z == 0 || z + 1 == q.tzn) st_dev(S.z + q.col + (T.z0 + z) * nxy, ur[z]);
        if (XF && q.xside >= 0) st_dev(xface_of(xf, S.team, 0, 0) + xfo + 8 * z, ur[z]);
      }
  }
  // the neighbours' u0 faces start loading into the u ring as soon as their
  // slots show that they are published (the set-up's x0 values there are used)
  ok &= team_sum_dev<3>(S, rank, red, acc3, rs, res_neighbours(g, tile, S.team, S.xcd_order, [&]() {
                          int tid_l = threadIdx.x, nxy_l = nxy;
                          asm volatile("" : "+v"(tid_l));
                          asm volatile("" : "+s"(nxy_l));
                          if constexpr (XF)
                            ring_dma<G>(g, q, lring, S.z, tid_l, nxy_l, xface_of(xf, S.team, 0, 0), tile);
                          else
                            ring_dma<G>(g, q, lring, S.z, tid_l, nxy_l);
                        }));
  stamp();
  const double bb = acc3[0];
  double gam = acc3[1], rr = acc3[2];

  float* ub[2] = {S.z, S.u1};
  float* wb[2] = {S.w0, S.w1};
  float* sb[2] = {S.s0, S.s1};
  int it = 0, status = kOk;
  if (!(ok && bb != 0.0 && rr > S.rtol2 * bb)) {
    __builtin_amdgcn_s_waitcnt(0);          // no solve: the u ring's loads end before LDS is reused
    __syncthreads();
  }
  if (ok && bb == 0.0) {
    if (q.own) {
#pragma unroll
      for (int z = 0; z < TZ; ++z)
        if (z < q.tzn) V.x[q.col + (T.z0 + z) * nxy] = 0.f;
    }
    xtop = 0.f;
    rr = 0.0;
  } else if (ok && rr > S.rtol2 * bb) {
    // ---------------- w0 = A u0
    if (q.own && q.bot_z) zlo[0] = ld_dev(ub[0] + q.col + (T.z0 - 1) * nxy);
    if (q.own && q.top_z) zhi[0] = ld_dev(ub[0] + q.col + T.z1 * nxy);
    __builtin_amdgcn_s_waitcnt(0);          // the u ring has landed
    __syncthreads();
    double acc1[1] = {0.0};
    // w0 / D on the tile's faces is published as each plane is done (no
    // global loads in the sweep, so the stores never hold up a wait)
    plane_sweep<G, 1, PZ>(g, q, lp, lring, [&](int, int z) { return ur[z]; }, zlo, zhi,
                   [&](int z, float* const* pl, const float* vzm, const float* vzp) {
                     const Nb n = faces_at<G>(la, q, z, sx, sy, sz);
                     const float w = apply_at(n, sx, sy, sz, ur[z], pl[0], q.oslot, G::PW, vzm[0], vzp[0]);
                     wr[z] = w * rcp<float>(n.D);
                     acc1[0] += (double)ur[z] * (double)w;
                     if (fedge || z == 0 || z + 1 == q.tzn) st_dev(wb[0] + q.col + (T.z0 + z) * nxy, wr[z]);
                     if (XF && q.xside >= 0) st_dev(xface_of(xf, S.team, 1, 0) + xfo + 8 * z, wr[z]);
                   });
    stamp();
    // the first iteration's halo rings (u0, w0/D; no s yet) start loading as
    // soon as the neighbours have published
    float* ring_u = lring;
    float* ring_w = lring + kResTZ * kRing;
    float* ring_s = lring + 2 * kResTZ * kRing;
    ok &= team_sum_dev<1>(S, rank, red, acc1, rs, res_neighbours(g, tile, S.team, S.xcd_order, [&]() {
                            int tid_l = threadIdx.x, nxy_l = nxy;
                            asm volatile("" : "+v"(tid_l));
                            asm volatile("" : "+s"(nxy_l));
                            // (u0 is in ring_u already)
                            if constexpr (XF)
                              ring_dma<G>(g, q, ring_w, wb[0], tid_l, nxy_l, xface_of(xf, S.team, 1, 0), tile);
                            else
                              ring_dma<G>(g, q, ring_w, wb[0], tid_l, nxy_l);
                          }));
    stamp();
    double a_cg = gam / acc1[0], b_cg = 0.0;
    int cur = 0;
    while (ok) {
      if (it >= S.max_iter) { status |= kNoConv; break; }
      // keep per-plane address arithmetic inside the loop (hoisting it for every
      // plane would exhaust the register file)
      int nxy_l = nxy;
      int col_l = q.col;
      asm volatile("" : "+s"(nxy_l));
      asm volatile("" : "+v"(col_l));
      // the tile's depth and first plane too: held constant, every plane's
      // comparisons and offsets would be computed once before the loop and
      // kept in scalar registers spilled to vector lanes, reloaded per plane
      ResPos ql = q;
      int z0_l = T.z0;
      asm volatile("" : "+s"(ql.tzn));
      asm volatile("" : "+s"(z0_l));
      const float a = (float)a_cg, b = (float)b_cg;
      const bool first = it == 0;
      // the neighbours' published u, w/D, s/D on the tile's ring are on their
      // way to LDS already (started inside the last reduction); the values
      // below and above the tile are loaded now and land while the registers
      // are updated
      const float* uo = ub[cur];
      const float* wo = wb[cur];
      const float* so = sb[cur];
      int tid_l = threadIdx.x;
      asm volatile("" : "+v"(tid_l));
      float zl[3] = {0.f, 0.f, 0.f}, zh[3] = {0.f, 0.f, 0.f};
      if (q.own && q.bot_z) {
        const int i = col_l + (T.z0 - 1) * nxy_l;
        zl[0] = ld_dev(uo + i); zl[1] = ld_dev(wo + i); zl[2] = first ? 0.f : ld_dev(so + i);
      }
      if (q.own && q.top_z) {
        const int i = col_l + T.z1 * nxy_l;
        zh[0] = ld_dev(uo + i); zh[1] = ld_dev(wo + i); zh[2] = first ? 0.f : ld_dev(so + i);
      }
      // elementwise updates: s = w + b s, p = u + b p, u -= a s in registers
      // (x += a p follows plane by plane in the sweep, where its memory
      // traffic hides behind the stencil's arithmetic). In the first
      // iteration b = 0 and s = 0, and p holds the finite x0, so the same
      // fused forms give s = w and p = u exactly.
#pragma unroll
      for (int z = 0; z < TZ; ++z) {
        const float s_ = fmaf(b, sr[z], wr[z]);
        const float p_ = fmaf(b, pr[z], ur[z]);
        pr[z] = p_;
        sr[z] = s_;
        ur[z] = fmaf(-a, s_, ur[z]);
      }
      // halo values of the new u from the neighbours' published u, w/D, s/D
      // (first iteration: b = 0 and the s values are zeros)
      auto unew = [&](float u_, float w_, float s_) { return fmaf(-a, fmaf(b, s_, w_), u_); };
      zlo[0] = unew(zl[0], zl[1], zl[2]);
      zhi[0] = unew(zh[0], zh[1], zh[2]);
      if (S.trace_detail) stamp();
      __builtin_amdgcn_s_waitcnt(0);        // the ring loads have reached LDS
      __syncthreads();
      // the ring's new u, in place
      // (every slot: slots past the tile's planes and outside the grid hold zeros)
#pragma unroll
      for (int e0 = 0; e0 < kResTZ * kRing; e0 += kResBlock) {
        const int e = e0 + tid_l;
        ring_u[e] = unew(ring_u[e], ring_w[e], ring_s[e]);
      }
      __syncthreads();
      if (S.trace_detail) stamp();
      double acc[3] = {0.0, 0.0, 0.0};
      // u, w/D, s/D on the tile's faces are published for the next iteration
      // as each plane is done. The other bank, written here, was last read by
      // the neighbours before the previous reduction, which this workgroup
      // has passed.
      float* uo_n = ub[cur ^ 1];
      float* wo_n = wb[cur ^ 1];
      float* so_n = sb[cur ^ 1];
      // x += a p of this iteration, plane by plane; each plane's x is loaded
      // two planes ahead of its update (only this workgroup touches its x).
      // x and the published faces go through buffer accesses: a lane offset
      // and a uniform plane offset, lanes off the grid (or, for the faces,
      // inside the tile) out of range.
      constexpr int kXAhead = 2;
      const __amdgpu_buffer_rsrc_t rx = vec_rsrc(V.x, g.ng);
      const __amdgpu_buffer_rsrc_t ru = vec_rsrc(uo_n, g.ng), rw = vec_rsrc(wo_n, g.ng), rs_ = vec_rsrc(so_n, g.ng);
      const unsigned vown = q.own ? 4u * (unsigned)col_l : kNoLane;
      const unsigned vedge = q.own && fedge ? 4u * (unsigned)col_l : kNoLane;
      // the compact x-edge columns of this iteration's bank: a lane offset on
      // the x-edge columns, constant offsets per vector and plane
      const __amdgpu_buffer_rsrc_t rxf = vec_rsrc(xf, XF ? 2LL * S.team * kXfTile : 0);
      const unsigned vxf =
          XF && q.own && q.xside >= 0 ? 4u * (unsigned)(xfo + (cur ^ 1) * S.team * kXfTile) : kNoLane;
      const int pbytes = 4 * nxy_l;
      float xq[kXAhead + 1];
#pragma unroll
      for (int z = 0; z < kXAhead; ++z) xq[z] = z < ql.tzn ? buf_ld(rx, vown, (z0_l + z) * pbytes) : 0.f;
      plane_sweep<G, 1, PZ>(g, ql, lp, ring_u, [&](int, int z) { return ur[z]; }, zlo, zhi,
                     [&](int z, float* const* pl, const float* vzm, const float* vzp) {
                       if (z + kXAhead < ql.tzn)
                         xq[(z + kXAhead) % (kXAhead + 1)] = buf_ld(rx, vown, (z0_l + z + kXAhead) * pbytes);
                       const Nb n = faces_at<G>(la, q, z, sx, sy, sz);
                       const float w = apply_at(n, sx, sy, sz, ur[z], pl[0], q.oslot, G::PW, vzm[0], vzp[0]);
                       wr[z] = w * rcp<float>(n.D);
                       const double ud = ur[z], Dd = n.D, rd = Dd * ud;
                       acc[0] += rd * ud;
                       acc[1] += (double)w * ud;
                       acc[2] += rd * rd;
                       const unsigned vf = (z == 0 || z + 1 == ql.tzn) ? vown : vedge;
                       const int so = (z0_l + z) * pbytes;
                       buf_st<kCpolSc1>(ru, vf, so, ur[z]);
                       buf_st<kCpolSc1>(rw, vf, so, wr[z]);
                       buf_st<kCpolSc1>(rs_, vf, so, sr[z]);
                       if (XF) {
                         buf_st<kCpolSc1>(rxf, vxf, 32 * z, ur[z]);
                         buf_st<kCpolSc1>(rxf, vxf, 4 * kXfCol + 32 * z, wr[z]);
                         buf_st<kCpolSc1>(rxf, vxf, 8 * kXfCol + 32 * z, sr[z]);
                       }
                       const float xn = fmaf(a, pr[z], xq[z % (kXAhead + 1)]);
                       buf_st(rx, vown, so, xn);
                       if (z == 0) xtop = xn;
                     });
      stamp();
      if (S.trace_detail) stamp();
      // the next iteration's halo rings start loading as soon as the
      // neighbours have published this sweep's faces
      ok &= team_sum_dev<3>(S, rank, red, acc, rs, res_neighbours(g, tile, S.team, S.xcd_order, [&]() {
                              int tid_r = threadIdx.x, nxy_r = nxy;
                              asm volatile("" : "+v"(tid_r));
                              asm volatile("" : "+s"(nxy_r));
                              if constexpr (XF) {
                                ring_dma<G>(g, q, ring_u, uo_n, tid_r, nxy_r, xface_of(xf, S.team, 0, cur ^ 1), tile);
                                ring_dma<G>(g, q, ring_w, wo_n, tid_r, nxy_r, xface_of(xf, S.team, 1, cur ^ 1), tile);
                                ring_dma<G>(g, q, ring_s, so_n, tid_r, nxy_r, xface_of(xf, S.team, 2, cur ^ 1), tile);
                              } else {
                                ring_dma<G>(g, q, ring_u, uo_n, tid_r, nxy_r);
                                ring_dma<G>(g, q, ring_w, wo_n, tid_r, nxy_r);
                                ring_dma<G>(g, q, ring_s, so_n, tid_r, nxy_r);
                              }
                            }));
      stamp();
      ++it;
      cur ^= 1;
      rr = acc[2];
      if (!(rr > S.rtol2 * bb)) break;
      const double gn = acc[0], dn = acc[1];
      b_cg = gn / gam;
      a_cg = gn / (dn - b_cg * gn / a_cg);
      gam = gn;
    }
    // the halo loads started in the last reduction land before LDS is reused
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }
  if (!(bb < INFINITY) || !(rr < INFINITY) || rr != rr) status |= kNonFinite;
  if (!ok) status |= kTimeout;

  // ---------------- epilogue: surface frame, checkpoint copy; for the gradient
  // the final x on the tile's faces is republished with device-scope stores
  if (q.own) {
    if (V.surf_out && T.z0 == 0) V.surf_out[q.col] = S.mode == kForward ? xtop : V.surf_scale * xtop;
    if (V.ckpt_out) {
      for (int z = 0; z < q.tzn; ++z) {
        const int i = q.col + (T.z0 + z) * nxy;
        V.ckpt_out[i] = V.x[i];
      }
    }
  }
  if (S.mode == kAdjoint && V.T_grad && ok) {
    // gradient: G_p -= sum_f s_f (a_q/(a_p+a_q))^2 (T_p-T_q)(mu_p-mu_q),
    // a_q/(a_p+a_q) = (1/a_p)/(1/a_p + 1/a_q) from the reciprocals in LDS
    float (&mcol)[TZ] = ur;                 // the solve is over: mu and T columns reuse u and p
    float (&tcol)[TZ] = pr;
#pragma unroll
    for (int z = 0; z < TZ; ++z) {
      const bool in = q.own && z < q.tzn;
      const int i = q.col + (T.z0 + z) * nxy;
      mcol[z] = in ? V.x[i] : 0.f;
      tcol[z] = in ? V.T_grad[i] : 0.f;
      if (in && (q.edge || z == 0 || z + 1 == q.tzn)) st_dev(V.x + i, mcol[z]);
    }
    double dummy[1] = {0.0};
    ok &= team_sum_dev<1>(S, rank, red, dummy, rs);
    float* ring_mu = lring;
    float* ring_T = lring + (size_t)kResTZ * kRing;
    fill_ring<G>(g, q, ring_mu, [&](int i) { return ld_dev(V.x + i); });
    fill_ring<G>(g, q, ring_T, [&](int i) { return V.T_grad[i]; });
    float glo[2] = {0.f, 0.f}, ghi[2] = {0.f, 0.f};
    if (q.own && q.bot_z) {
      glo[0] = ld_dev(V.x + q.col + (T.z0 - 1) * nxy);
      glo[1] = V.T_grad[q.col + (T.z0 - 1) * nxy];
    }
    if (q.own && q.top_z) {
      ghi[0] = ld_dev(V.x + q.col + T.z1 * nxy);
      ghi[1] = V.T_grad[q.col + T.z1 * nxy];
    }
    __syncthreads();
    plane_sweep<G, 2, 1>(g, q, lp, lring, [&](int k, int z) { return k == 0 ? mcol[z] : tcol[z]; }, glo, ghi,
                   [&](int z, float* const* pl, const float* vzm, const float* vzp) {
                     const float* plz = la + (z + 1) * G::PL + q.oslot;
                     const double ia = plz[0];
                     const double m = mcol[z], t = tcol[z];
                     double qa[6], dm[6], dT[6];
                     qa[0] = plz[-1]; qa[1] = plz[1];
                     qa[2] = plz[-G::PW]; qa[3] = plz[G::PW];
                     qa[4] = plz[-G::PL]; qa[5] = plz[G::PL];
                     dm[0] = m - (double)pl[0][q.oslot - 1]; dT[0] = t - (double)pl[1][q.oslot - 1];
                     dm[1] = m - (double)pl[0][q.oslot + 1]; dT[1] = t - (double)pl[1][q.oslot + 1];
                     dm[2] = m - (double)pl[0][q.oslot - G::PW]; dT[2] = t - (double)pl[1][q.oslot - G::PW];
                     dm[3] = m - (double)pl[0][q.oslot + G::PW]; dT[3] = t - (double)pl[1][q.oslot + G::PW];
                     dm[4] = m - (double)vzm[0]; dT[4] = t - (double)vzm[1];
                     dm[5] = m - (double)vzp[0]; dT[5] = t - (double)vzp[1];
                     const double sf[6] = {(double)sx, (double)sx, (double)sy, (double)sy, (double)sz, (double)sz};
                     double gsum = 0.0;
#pragma unroll
                     for (int f = 0; f < 6; ++f) {
                       const double w = ia / (ia + qa[f]);
                       gsum += sf[f] * (w * w) * (dT[f] * dm[f]);
                     }
                     const int i = q.col + (T.z0 + z) * nxy;
                     S.G[i] = S.G[i] - gsum;
                   });
  }

  stamp();
  if (publish) {
    // The solution was stored with ordinary stores (the last part after the
    // final reduction): make it visible to the whole team before a following
    // step in the same launch reads its neighbours' cells. The barrier takes
    // the next epoch of the step's sequence, so that it and the reductions
    // before and after it (the caller starts the next step from epoch_end)
    // alternate between the two slot banks.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    double none[1] = {0.0};
    if (!team_sum_dev<1>(S, rank, red, none, rs)) status |= kTimeout;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  const double relres = bb > 0.0 ? sqrt(rr / bb) : 0.0;
  if (V.out_iters && rank == 0 && threadIdx.x == 0) {
    V.out_iters[0] = it;
    V.out_relres[0] = relres;
    V.out_status[0] = status;
  }
  return StepResult{it, status, relres, red};
}

template <int TXC>
__global__ void __launch_bounds__(kResBlock, 1) resident_step_kernel(StepArgs<float> S) {
  extern __shared__ __align__(16) unsigned char dsm[];
  resident_step<TXC, kResPZ, true>(S, step_var(S), blockIdx.x, dsm, false);
}

}  // namespace nh
