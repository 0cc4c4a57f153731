// The batched-ensemble kernel: many Gray-Scott instances stepped by one
// persistent kernel with the same stage tiles (stage.h) as the single-grid
// path.
#include "stage.h"

#include <type_traits>

namespace hode {

namespace {

constexpr int kEnsThreads = 64 * kEnsNW;
// LDS of the ensemble's largest tile: the row slots of two-row strips of
// 16-byte lanes, and the x-halo cells of up to four-row strips of 8-byte
// cells (every tile checks its own size against this).
constexpr int kEnsSmem = 2 * 2 * (2 * kEnsNW + 2) * 64 * 16 + 2 * 2 * 2 * (kEnsNW * 4) * 8;

// ---- the persistent ensemble kernel -------------------------------------------
// One launch steps every unfinished instance for up to `rounds` attempts in
// lock step (by default the whole integration: the launch ends when every
// instance is done): each round runs the six stage phases of a Dopri5
// attempt and a control phase, with a grid-wide barrier after each.  A stage phase is a
// pool of tiles (instance, rows, planes) covering every instance; the host
// deals the instances to eight queues, one per XCD, and a workgroup claims
// tiles from its own XCD's queue first (neighbouring tiles, whose halo rows
// overlap, then share an L2) and from the others once it is empty, so each
// phase is balanced dynamically.  The control phase runs each instance's
// step controller on one workgroup.  Instances that are done, or reached
// the launch's pause point, skip their tiles and control; the host then
// relaunches with the instances still running, and a resumed instance skips
// stage 1 (its k1 is in the first-same-as-last slot), so pausing changes no
// result.  The grid barrier is a 64-bit arrival counter with device-scope
// release/acquire; the grid is sized from the occupancy so every workgroup
// is resident at once, and a barrier that waits longer than spin_limit polls
// flags an error on which every workgroup leaves.  The claim counters of the
// stage phases and the per-round count of running instances come in two
// alternating sets, each cleared by workgroup 0 once every workgroup has
// passed a barrier after its last use, so a launch of any length needs no
// further bookkeeping memory.

__device__ inline bool ens_error(const EnsSched& s) {
  return __hip_atomic_load(s.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// Two-level arrival: a workgroup counts itself on its XCD's line (workgroups
// are dealt round-robin to the 8 XCDs), the last arrival of each XCD counts
// the XCD on the global line, and every workgroup waits for all XCDs there:
// 8 arrival atomics per barrier on the global line instead of one per
// workgroup.
__device__ inline void grid_sync(const EnsSched& s, uint64_t& gen) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();  // release this workgroup's outputs
    const uint32_t x = blockIdx.x & 7;
    const uint64_t per_xcd = (gridDim.x - x + 7) / 8;  // workgroups of this XCD
    const uint64_t mine = atomicAdd((unsigned long long*)(s.xbar + 16 * x), 1ull) + 1;
    if (mine == (gen + 1) * per_xcd) atomicAdd((unsigned long long*)s.bar, 1ull);
    const uint64_t target = (gen + 1) * (uint64_t)(gridDim.x < 8 ? gridDim.x : 8);
    int64_t spins = 0;
    while (__hip_atomic_load(s.bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(2);
      if (++spins > s.spin_limit) {
        atomicExch(s.error, 1u);
        break;
      }
      if ((spins & 255) == 0 && ens_error(s)) break;
    }
    __threadfence();  // acquire everyone's outputs
  }
  __syncthreads();
  ++gen;
}

// The arguments of a device function arrive in vector registers; the launch
// description is the same for every lane, so it is copied word by word
// through the first lane into scalar registers (as a kernel argument would
// be), which keeps the array pointers and grid constants out of the vector
// register budget of the stage loop.
template <typename S>
__device__ inline S uniform_copy(const S& src) {
  static_assert(sizeof(S) % 4 == 0, "word copy");
  uint32_t w[sizeof(S) / 4];
  __builtin_memcpy(w, &src, sizeof(S));
#pragma unroll
  for (int i = 0; i < (int)(sizeof(S) / 4); ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
  S out;
  __builtin_memcpy(&out, w, sizeof(S));
  return out;
}

// Rows per wave of the ensemble's tiles: narrow rows (few cells per lane)
// take more rows per wave, so each plane step still has about 16 bytes of
// state per lane and field in flight, except where that would exceed the
// persistent kernel's register budget (stage 6, the widest, keeps half).
// The host cuts tiles into row chunks of the non-stage-6 pass height, which
// the stage-6 height divides.
template <typename T, int KIND, int VW>
constexpr int ens_rows() {
  constexpr int full = (int)(16 / sizeof(T)) / VW;
  constexpr int r = KIND == K_D6 ? full / 2 : full;
  return r < 1 ? 1 : r;
}

// Not inlined: each stage variant keeps its own register allocation, so the
// persistent kernel's budget is the largest single stage, not their union.
// SEG > 1: segmented rows (16-byte lanes, one whole row per segment of
// 64/SEG lanes; see stage_tile).
template <typename T, int KIND, int VW, int SEG = 1>
__device__ __noinline__ void ens_tile_vw(EnsInst* I, char* smem, int y0, int y1, int z0, int z1) {
  // segmented rows: two register rows of SEG rows each (stage 6, the widest, one)
  constexpr int RY = SEG == 1 ? ens_rows<T, KIND, VW>() : (KIND == K_D6 ? 1 : 2);
  constexpr int TY = kEnsNW * RY * SEG;
  static_assert(tile_smem<T, VW, RY, kEnsNW, SEG>() <= kEnsSmem, "the tile fits the kernel's LDS");
  const GSLaunch a = uniform_copy(I->a);
  DevCtrl* c = uniform_copy(&I->ctrl);
  y0 = __builtin_amdgcn_readfirstlane(y0);
  y1 = __builtin_amdgcn_readfirstlane(y1);
  z0 = __builtin_amdgcn_readfirstlane(z0);
  z1 = __builtin_amdgcn_readfirstlane(z1);
  const int nx = (a.N + 64 * VW - 1) / (64 * VW);
  for (int ty = y0 / TY; ty * TY < y1; ++ty)
    for (int tx = 0; tx < nx; ++tx) stage_tile<T, KIND, RY, VW, SEG, kEnsNW>(a, c, smem, tx, ty, z0, z1);
}

template <typename T, int KIND>
__device__ void ens_tile(EnsInst* I, char* smem, const EnsTile& t) {
  constexpr int VF = (int)(16 / sizeof(T));  // cells per 16-byte lane
  switch (I->seg) {
    case 2: return ens_tile_vw<T, KIND, VF, 2>(I, smem, t.y0, t.y1, t.z0, t.z1);
    case 3: return ens_tile_vw<T, KIND, VF, 3>(I, smem, t.y0, t.y1, t.z0, t.z1);
    case 4: return ens_tile_vw<T, KIND, VF, 4>(I, smem, t.y0, t.y1, t.z0, t.z1);
    case 5: return ens_tile_vw<T, KIND, VF, 5>(I, smem, t.y0, t.y1, t.z0, t.z1);
    case 6: return ens_tile_vw<T, KIND, VF, 6>(I, smem, t.y0, t.y1, t.z0, t.z1);
    case 8: return ens_tile_vw<T, KIND, VF, 8>(I, smem, t.y0, t.y1, t.z0, t.z1);
    case 10: return ens_tile_vw<T, KIND, VF, 10>(I, smem, t.y0, t.y1, t.z0, t.z1);
    case 16: return ens_tile_vw<T, KIND, VF, 16>(I, smem, t.y0, t.y1, t.z0, t.z1);
    default: break;
  }
  if constexpr (sizeof(T) == 4) {
    if (I->vw == 4) return ens_tile_vw<T, KIND, 4>(I, smem, t.y0, t.y1, t.z0, t.z1);
    if (I->vw == 2) return ens_tile_vw<T, KIND, 2>(I, smem, t.y0, t.y1, t.z0, t.z1);
  } else {
    if (I->vw == 2) return ens_tile_vw<T, KIND, 2>(I, smem, t.y0, t.y1, t.z0, t.z1);
  }
  ens_tile_vw<T, KIND, 1>(I, smem, t.y0, t.y1, t.z0, t.z1);
}

// An instance takes part in a round's phases while it is not done and below
// its pause point (both change only in the control phase).
__device__ inline bool ens_running(const EnsInst* I) {
  return !__hip_atomic_load(&I->ctrl.done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &&
         __hip_atomic_load(&I->ctrl.attempts, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < I->pause_at;
}

// Tiles of one instance for a target of `target` cells per tile: row chunks
// of one tile pass, plane chunks of zc planes (the instance's own zc if set,
// else sized from the target, at least 4 planes).
__device__ inline void ens_tile_grid(const EnsInst* I, double target, int* ny, int* nz) {
  const int N = I->a.N, rows = I->rows;
  int zc = I->zc_fix > 0 ? I->zc_fix : (int)floor(target / ((double)N * rows) + 0.5);
  zc = max(I->zc_fix > 0 ? 1 : 4, min(N, zc));
  *ny = (N + rows - 1) / rows;
  *nz = (N + zc - 1) / zc;
}

// Re-tiling (workgroup 0, all its threads, between two grid barriers, with
// the tile LDS free): the instances still running, in the dealing order of
// s.order (largest work estimate first), are cut into tiles sized so a phase
// again has about kTilesPerWorkgroup tiles per workgroup, and dealt onto the
// eight per-XCD queues, each to the least-loaded one, as the host does before
// the launch.  As instances finish, the remaining ones are cut finer, so the
// phases keep every workgroup busy.  Per-instance lists live in the tile LDS
// (at most kRetileMaxInst instances).
__device__ void ens_retile(EnsInst* __restrict__ inst, const EnsSched& s, const EnsParams& prm, char* smem) {
  int* act = reinterpret_cast<int*>(smem);
  float* w = reinterpret_cast<float*>(smem + 4 * kRetileMaxInst);
  int* base = reinterpret_cast<int*>(smem + 8 * kRetileMaxInst);
  uint8_t* qk = reinterpret_cast<uint8_t*>(smem + 12 * kRetileMaxInst);
  static_assert(13 * kRetileMaxInst <= kEnsSmem, "re-tiling lists fit the tile LDS");
  __shared__ int s_cnt[kEnsThreads], s_qoff[9], s_m;
  __shared__ double s_cells[kEnsThreads], s_target;
  const int n = prm.n_inst, tid = threadIdx.x;
  __syncthreads();
  // running instances in dealing order: contiguous chunks per thread, then
  // an exclusive scan of the chunk counts
  const int per = (n + kEnsThreads - 1) / kEnsThreads, j0 = min(n, tid * per), j1 = min(n, j0 + per);
  int cnt = 0;
  double cells = 0;
  for (int j = j0; j < j1; ++j) {
    const EnsInst* I = &inst[s.order[j]];
    if (ens_running(I)) {
      ++cnt;
      cells += (double)I->a.n3;
    }
  }
  s_cnt[tid] = cnt;
  s_cells[tid] = cells;
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    double cs = 0;
    for (int t = 0; t < kEnsThreads; ++t) {
      const int c0 = s_cnt[t];
      s_cnt[t] = acc;
      acc += c0;
      cs += s_cells[t];
    }
    s_m = acc;
    s_target = fmax(4096.0, cs / (kTilesPerWorkgroup * gridDim.x));
  }
  __syncthreads();
  {
    int k = s_cnt[tid];
    for (int j = j0; j < j1; ++j) {
      const int i = s.order[j];
      const EnsInst* I = &inst[i];
      if (ens_running(I)) {
        act[k] = i;
        w[k] = I->weight;
        ++k;
      }
    }
  }
  __syncthreads();
  const int m = s_m;
  const double target = s_target;
  for (int k = tid; k < m; k += kEnsThreads) {
    int ny, nz;
    ens_tile_grid(&inst[act[k]], target, &ny, &nz);
    base[k] = ny * nz;  // tile count for now
  }
  __syncthreads();
  if (tid == 0) {
    double load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int qt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = 0; k < m; ++k) {
      int x = 0;
      for (int y = 1; y < 8; ++y)
        if (load[y] < load[x]) x = y;
      qk[k] = (uint8_t)x;
      load[x] += w[k];
      qt[x] += base[k];
    }
    int run[8], acc = 0;
    for (int x = 0; x < 8; ++x) {
      s_qoff[x] = run[x] = acc;
      acc += qt[x];
    }
    s_qoff[8] = acc;
    for (int k = 0; k < m; ++k) {
      const int nt = base[k];
      base[k] = run[qk[k]];
      run[qk[k]] += nt;
    }
    if (acc > prm.tiles_cap) atomicExch(s.error, 3u);  // the host sizes the buffer for the finest cut
  }
  __syncthreads();
  if (s_qoff[8] > prm.tiles_cap) return;
  if (tid <= 8) s.qoff[tid] = s_qoff[tid];
  // plane-chunk-major, row-chunk-minor (tiles sharing halo rows adjacent)
  for (int k = tid; k < m; k += kEnsThreads) {
    const int i = act[k];
    EnsInst* I = &inst[i];
    const int N = I->a.N, rows = I->rows;
    int ny, nz;
    ens_tile_grid(I, target, &ny, &nz);
    int t = base[k];
    for (int kz = 0; kz < nz; ++kz) {
      const int z0 = (int)((int64_t)N * kz / nz), z1 = (int)((int64_t)N * (kz + 1) / nz);
      for (int ky = 0; ky < ny; ++ky) s.tiles[t++] = EnsTile{i, rows * ky, min(N, rows * (ky + 1)), z0, z1, 0};
    }
    I->ntiles = ny * nz;
  }
}

template <typename T>
__global__ __launch_bounds__(kEnsThreads, 1) void ens_kernel(EnsInst* __restrict__ inst, const EnsSched s) {
  __shared__ __align__(16) char smem[kEnsSmem];
  __shared__ int s_claim, s_run, s_last;
  const EnsParams prm = *s.params;
  const int xcd = blockIdx.x & 7;  // workgroups are dealt round-robin to the 8 XCDs
  uint64_t gen = 0;
  int phase = 0;

  // one stage phase over every queue's tiles; false once an error is flagged
  auto stage_phase = [&](auto kind, int round) -> bool {
    constexpr int K = decltype(kind)::value;
    if (blockIdx.x == 0 && threadIdx.x < 8) {
      // the other set of claim counters was last used by the previous phase,
      // which every workgroup has left (barrier): clear it for the next
      __hip_atomic_store(s.qctr + ((phase + 1) & 1) * 8 + threadIdx.x, 0u, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
      // the other round's count of running instances was last read right
      // after the barrier that ended that round, before this round's first
      // phase: clear it from the second phase of this round on
      if (K == K_D3 && threadIdx.x == 0)
        __hip_atomic_store(s.live + ((round + 1) & 1), 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    for (int q = 0; q < 8; ++q) {
      const int x = (xcd + q) & 7;
      const int base = s.qoff[x], cnt = s.qoff[x + 1] - base;
      uint32_t* ctr = s.qctr + (phase & 1) * 8 + x;
      for (;;) {
        if (threadIdx.x == 0) {
          int t = cnt;
          if ((int)__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < cnt) t = (int)atomicAdd(ctr, 1u);
          int run = 0;
          if (t < cnt) {
            const EnsInst* I = &inst[s.tiles[base + t].inst];
            run = K == K_D1 ? (!I->k1_valid && ens_running(I)) : ens_running(I);
          }
          s_claim = t;
          s_run = run;
        }
        __syncthreads();
        const int t = s_claim, run = s_run;
        __syncthreads();
        if (t >= cnt) break;
        if (run) {
          const EnsTile tl = s.tiles[base + t];
          EnsInst* I = &inst[tl.inst];
          ens_tile<T, K>(I, smem, tl);
          if constexpr (K == K_D7) {
            // the workgroup that finishes the instance's last tile of the
            // attempt runs its step control: the error maxima of every tile
            // are device-scope atomics made before their count
            __syncthreads();
            if (threadIdx.x == 0) {
              __threadfence();
              s_last = atomicAdd(&I->last_done, 1u) + 1 == (uint32_t)I->ntiles;
            }
            __syncthreads();
            if (s_last) {
              if (threadIdx.x == 0) {
                __threadfence();
                __hip_atomic_store(&I->last_done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              }
              ctrl_step(&I->ctrl);
              if (threadIdx.x == 0 && ens_running(I)) atomicAdd(&s.live[round & 1], 1u);
            }
          }
        }
      }
    }
    ++phase;
    grid_sync(s, gen);
    return !ens_error(s);
  };

  if (prm.first_d1 && !stage_phase(std::integral_constant<int, K_D1>(), 0)) return;
  int retile_at = prm.retile_at;
  for (int r = 0; r < prm.rounds; ++r) {
    if (!stage_phase(std::integral_constant<int, K_D2>(), r)) return;
    if (!stage_phase(std::integral_constant<int, K_D3>(), r)) return;
    if (!stage_phase(std::integral_constant<int, K_D4>(), r)) return;
    if (!stage_phase(std::integral_constant<int, K_D5>(), r)) return;
    if (!stage_phase(std::integral_constant<int, K_D6>(), r)) return;
    // (the last phase also ran every instance's step control)
    if (!stage_phase(std::integral_constant<int, K_D7>(), r)) return;
    // every instance finished or paused: leave early (uniform: all read after the barrier)
    const int live = (int)__hip_atomic_load(&s.live[r & 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (live == 0) return;
    // half of the instances of the last tiling are done: cut the rest finer
    if (live <= retile_at) {
      if (blockIdx.x == 0) ens_retile(inst, s, prm, smem);
      grid_sync(s, gen);
      if (ens_error(s)) return;
      retile_at = live / 2;
    }
  }
}

}  // namespace

hipError_t launch_ensemble(int dtype, EnsInst* inst, EnsSched s, int nwg, hipStream_t st) {
  if (nwg < 1) return hipErrorInvalidValue;
  if (dtype == 1) ens_kernel<float><<<nwg, kEnsThreads, 0, st>>>(inst, s);
  else ens_kernel<double><<<nwg, kEnsThreads, 0, st>>>(inst, s);
  return hipGetLastError();
}

int ensemble_blocks_per_cu(int dtype) {
  int n = 0;
  hipError_t e = dtype == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, ens_kernel<float>, kEnsThreads, 0)
                            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, ens_kernel<double>, kEnsThreads, 0);
  return e == hipSuccess ? n : 0;
}

}  // namespace hode
