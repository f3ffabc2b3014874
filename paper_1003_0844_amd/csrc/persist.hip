// The whole grid call (Sec. VI A-B: sky preparation, both FFT passes, the F
// combination and the output) in one launch of a persistent kernel.
//
// The host lays the call out as a queue of tiles (PersistArgs, internal.h):
// for every batch of sky positions its set-up, record and coefficient tiles,
// for every node its R first-pass tiles and its R second-pass tiles, in an
// order where every tile depends only on tiles before it.  Each workgroup
// claims the next tile from a global counter, waits until what the tile
// reads is complete, runs it with the same tile functions as the
// launch-per-pass kernels (tiles.h), and counts it complete.  A workgroup
// claims tiles only while it runs, and a tile's dependencies lie earlier in
// the queue, so every wait ends (by induction over the queue) whether or not
// all workgroups are resident at once.  Each wait is also bounded in wall-clock
// time: past spin_ticks it sets the sticky error flag and every workgroup
// leaves the queue, so the kernel ends in any case.
//
// Dependencies (completion counters, cnt):
//   set-up of batch b      after batch b-2 (same sky set) has finished pass 2
//   record / coefficient   after the set-up of b
//   pass 1 of node n       after all record tiles of its batch, and after
//                          pass 2 of node n - nslots (the spill slot's last user)
//   pass 2 of node n       after pass 1 of n and the coefficients of its batch
// Completion is published with an agent-scope release (writer) and observed
// with an agent-scope acquire (reader): the workgroups of one dependency run
// on different XCDs, whose L2 caches are not coherent with each other.
//
// Pass 2 of node n interleaves with pass 1 of node n + L in the queue (L =
// nslots - 2, chosen by the host), so the spill of a node is read back while
// at most nslots nodes' spill is live.
#include "tiles.h"

namespace {

constexpr int PB = 256;   // threads per workgroup
constexpr int PC = 4096;  // first-pass length
constexpr int P_LDS = lds_slots(PC, 1);
static_assert(lds_slots(256, 16) == P_LDS && lds_slots(64, 64) == P_LDS && lds_slots(1024, 4) == P_LDS,
              "second-pass tiles with R x B2 = 4096 use the first pass's LDS");

// counters: per batch b at 4 b: set-up, record tiles, coefficients, pass-2
// tiles; per node n at 4 nbatch + 3 n: pass-1 tiles, pass-2 arrivals (max
// mode), pass-2 tiles
__device__ __forceinline__ uint32_t* batch_cnt(const PersistArgs& a, int b, int which) { return a.cnt + 4 * b + which; }
__device__ __forceinline__ uint32_t* node_cnt(const PersistArgs& a, int n, int which) {
  return a.cnt + 4 * (int64_t)a.nbatch + 3 * (int64_t)n + which;
}

__device__ __forceinline__ uint32_t load_cnt(const uint32_t* c) {
  return __hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait (one thread) until *c >= target; false if the wait outlived spin_ticks
// or another workgroup has given up.
__device__ bool wait_ge(const PersistArgs& a, const uint32_t* c, uint32_t target) {
  if (load_cnt(c) >= target) return true;
  const long long t0 = wall_clock64();
  for (;;) {
    __builtin_amdgcn_s_sleep(2);
    if (load_cnt(c) >= target) return true;
    if (load_cnt(a.error) != 0u) return false;
    if ((uint64_t)(wall_clock64() - t0) > a.spin_ticks) {
      __hip_atomic_fetch_or(a.error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
  }
}

// Publish one completion (one thread, after a workgroup barrier): everything
// the workgroup wrote becomes visible to the acquirers of *c.  The explicit
// wait after the fence keeps the L2 write-back complete before the count: at
// the head of the claim loop, with the previous tile's stores still in flight
// on the back edge, the compiler omits the wait the fence implies.
__device__ __forceinline__ void release_agent() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __builtin_amdgcn_s_waitcnt(0);
}
__device__ __forceinline__ void signal(uint32_t* c, uint32_t v = 1u) {
  release_agent();
  __hip_atomic_fetch_add(c, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

// A flag that thread 0 left in LDS, read as a wave-uniform value: the branch
// on it is a scalar branch, so every lane of a wave takes it together.
__device__ __forceinline__ bool uniform_flag(const int& v) { return __builtin_amdgcn_readfirstlane(v) != 0; }

__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const int hi = __builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// ---- tiles ----
__device__ __forceinline__ void sky_prep_tile(const SegDev& sg, const PBatch& bt, const PersistArgs& a, int t) {
  const int g = t / bt.nblk, blk = t - g * bt.nblk;
  const int s0 = g * SKY_GROUP;
  const int ng = min(SKY_GROUP, bt.nsky - s0);
  const int64_t qstride = (int64_t)sg.R * sg.Ceff;
  const SkyConst* skies = a.sky[bt.set] + s0;
  Quad<float>* out = (Quad<float>*)a.quads[bt.set] + (int64_t)s0 * qstride;
  const int64_t p0 = (int64_t)blk * PB * PREP_POS + threadIdx.x;
#pragma unroll 1
  for (int i = 0; i < PREP_POS; ++i) {
    const int64_t pos = p0 + (int64_t)i * PB;
    if (sg.interp == 0) sky_prep_pos<float, 0>(sg, skies, ng, pos, out, qstride);
    else if (sg.interp == 1) sky_prep_pos<float, 1>(sg, skies, ng, pos, out, qstride);
    else sky_prep_pos<float, 2>(sg, skies, ng, pos, out, qstride);
  }
}

template <int R, int MODE>
__device__ __forceinline__ void pass2_of(const SegDev& sg, const PersistArgs& a, const PSegTw& tw, const PBatch& bt,
                                         int n, int cb, lds_t<Pair<float>>* lds) {
  const NodeDev node = a.nodes[n];
  const int slot = n % a.nslots;
  pass2_tile<float, R, MODE>(sg, (const Pair<float>*)a.spill + (int64_t)slot * a.slot_elems, node,
                             a.coef[bt.set][node.sky], (const cpx<float>*)tw.twR, a.out, cb,
                             a.part + (int64_t)slot * 1024, lds);
}

template <bool BLK>
__device__ __forceinline__ void pass1_of(const SegDev& sg, const PersistArgs& a, const PSegTw& tw, const PBatch& bt,
                                         int n, int r, lds_t<Pair<float>>* lds) {
  const int slot = n % a.nslots;
  pass1_tile<float, PC, BLK>(sg, (const Quad<float>*)a.quads[bt.set], (int64_t)sg.R * sg.Ceff, a.sky[bt.set],
                             a.nodes[n], r, (const cpx<float>*)tw.twC, (const cpx<float>*)tw.twlo,
                             (const cpx<float>*)tw.twhi, (Pair<float>*)a.spill + (int64_t)slot * a.slot_elems,
                             lds);
}

template <int MODE>
__global__ void __launch_bounds__(PB, 3) k_persist(PersistArgs a) {
  __shared__ lds_t<Pair<float>> lds[P_LDS];
  __shared__ unsigned long long s_item;
  __shared__ int s_ok, s_last;
  const int tid = threadIdx.x;
  // Control flow: every branch that decides which barrier a thread reaches next
  // is taken on a wave-uniform value (the claimed item, or a flag thread 0 left
  // in LDS, read with readfirstlane), and every thread-0 block is followed by a
  // barrier before such a branch.  With a thread-0 block in front of the loop
  // latch (a completion signalled at the end of a tile) and another behind it
  // (the claim), the compiler may merge the two tests of tid == 0 and send
  // threads 1.. straight back to the barrier after the claim while thread 0's
  // lane waits outside that inner loop: the workgroup would run the same tile
  // over and over and never claim another.  So a tile's completion is counted
  // by thread 0 in the block that claims the next tile (or after the loop):
  // pend_rel / pend_add name the counters, set alike in every thread.
  uint32_t* pend_rel = nullptr;  // published with a release
  uint32_t* pend_add = nullptr;  // counted without one (a count the host schedule only reads in order)
  for (;;) {
    if (tid == 0) {
      if (pend_rel) signal(pend_rel);
      if (pend_add) __hip_atomic_fetch_add(pend_add, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_item = atomicAdd(a.head, 1ull);
    }
    pend_rel = pend_add = nullptr;
    __syncthreads();
    const int64_t item = uniform64((int64_t)s_item);
    if (item >= a.nitems) break;
    const PUnit u = a.units[item / PUNIT];
    const int tile = u.sub * PUNIT + (int)(item % PUNIT);

    if (u.kind == PU_SKY) {
      const int b = u.id;
      const PBatch bt = a.batches[b];
      const SegDev& sg = a.segs[bt.seg];
      const int ntiles = bt.nprep + 2;  // set-up, records, coefficients
      if (tile >= ntiles) {
        __syncthreads();  // s_item is read by every thread before the next claim
        continue;
      }
      if (tid == 0) {
        bool ok;
        if (tile == 0) {
          ok = b < 2 || wait_ge(a, batch_cnt(a, b - 2, 3), (uint32_t)(a.batches[b - 2].nnode * a.segs[a.batches[b - 2].seg].R));
        } else {
          ok = wait_ge(a, batch_cnt(a, b, 0), 1u);
        }
        if (ok) acquire();
        s_ok = ok;
      }
      __syncthreads();
      if (!uniform_flag(s_ok)) break;
      if (tile == 0) {
        if (tid < bt.nsky)
          a.sky[bt.set][tid] = sky_setup_one(a.sky_ad[2 * (bt.sky0 + tid)], a.sky_ad[2 * (bt.sky0 + tid) + 1], sg.geo);
      } else if (tile <= bt.nprep) {
        sky_prep_tile(sg, bt, a, tile - 1);
      } else {
        if (tid < bt.nsky) a.coef[bt.set][tid] = sky_coef_one(a.sky[bt.set][tid], sg.mom, sg.sigma2);
      }
      __syncthreads();
      pend_rel = batch_cnt(a, b, tile == 0 ? 0 : (tile <= bt.nprep ? 1 : 2));
      continue;
    }

    const int n = u.id;
    const int b = a.node_batch[n];
    const PBatch bt = a.batches[b];
    const SegDev& sg = a.segs[bt.seg];
    const PSegTw tw = a.tw[bt.seg];
    const int R = sg.R;
    if (u.kind == PU_P1) {
      if (tid == 0) {
        bool ok = wait_ge(a, batch_cnt(a, b, 1), (uint32_t)bt.nprep);
        if (ok && n >= a.nslots) {
          const int m = n - a.nslots;
          ok = wait_ge(a, node_cnt(a, m, 2), (uint32_t)a.segs[a.batches[a.node_batch[m]].seg].R);
        }
        if (ok) acquire();
        s_ok = ok;
      }
      __syncthreads();
      if (!uniform_flag(s_ok)) break;
      if (R > 128) pass1_of<true>(sg, a, tw, bt, n, tile, lds);  // the spill layout of pass 2's B2
      else pass1_of<false>(sg, a, tw, bt, n, tile, lds);
      __syncthreads();
      pend_rel = node_cnt(a, n, 0);
      continue;
    }

    // pass 2, column block `tile` of node n
    if (tid == 0) {
      bool ok = wait_ge(a, node_cnt(a, n, 0), (uint32_t)R);
      if (ok) ok = wait_ge(a, batch_cnt(a, b, 2), 1u);
      if (ok) acquire();
      s_ok = ok;
    }
    __syncthreads();
    if (!uniform_flag(s_ok)) break;
    switch (R) {
      case 64: pass2_of<64, MODE>(sg, a, tw, bt, n, tile, lds); break;
      case 128: pass2_of<128, MODE>(sg, a, tw, bt, n, tile, lds); break;
      case 256: pass2_of<256, MODE>(sg, a, tw, bt, n, tile, lds); break;
      case 512: pass2_of<512, MODE>(sg, a, tw, bt, n, tile, lds); break;
      default: pass2_of<1024, MODE>(sg, a, tw, bt, n, tile, lds); break;
    }
    __syncthreads();
    if constexpr (MODE == 1) {
      // the last column block of the node to arrive reduces its partials
      if (tid == 0) {
        release_agent();
        const uint32_t old = __hip_atomic_fetch_add(node_cnt(a, n, 1), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_last = old + 1u == (uint32_t)R;
        if (s_last) acquire();
      }
      __syncthreads();
      if (uniform_flag(s_last) && tid < 64) {
        const MaxPartial* p = a.part + (int64_t)(n % a.nslots) * 1024;
        double best = -1.0;
        int64_t bk = INT64_MAX;
        for (int i = tid; i < R; i += 64) {
          const MaxPartial q = p[i];
          if (q.F > best || (q.F == best && q.k < bk)) {
            best = q.F;
            bk = q.k;
          }
        }
        wave_argmax(best, bk);
        if (tid == 0) {
          const int row = a.nodes[n].row;
          ((float*)a.out.Fmax)[row] = (float)best;
          a.out.kmax[row] = bk;
        }
      }
      __syncthreads();
    }
    pend_rel = node_cnt(a, n, 2);
    pend_add = batch_cnt(a, b, 3);
  }
  // the last tile's completion (the loop ends at the claim after it, or on an error)
  if (tid == 0) {
    if (pend_rel) signal(pend_rel);
    if (pend_add) __hip_atomic_fetch_add(pend_add, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ void k_persist_zero(uint32_t* __restrict__ cnt, int64_t n32, unsigned long long* __restrict__ head) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n32) cnt[i] = 0u;
  if (i == 0) *head = 0ull;
}

}  // namespace

namespace fsk {

int persistent_blocks(int mode) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  hipError_t e;
  if (mode == 0) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_persist<0>, PB, 0);
  else if (mode == 1) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_persist<1>, PB, 0);
  else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_persist<2>, PB, 0);
  if (e != hipSuccess || per <= 0) return 0;
  return per * cus;
}

hipError_t persist_zero(uint32_t* cnt, int64_t n32, unsigned long long* head, hipStream_t st) {
  const int64_t n = n32 > 1 ? n32 : 1;
  hipLaunchKernelGGL(k_persist_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, cnt, n32, head);
  return hipGetLastError();
}

hipError_t grid_persistent(const PersistArgs& a, int mode, int blocks, hipStream_t st) {
  if (blocks <= 0) return hipErrorInvalidValue;
  if (mode == 0) hipLaunchKernelGGL(k_persist<0>, dim3(blocks), dim3(PB), 0, st, a);
  else if (mode == 1) hipLaunchKernelGGL(k_persist<1>, dim3(blocks), dim3(PB), 0, st, a);
  else hipLaunchKernelGGL(k_persist<2>, dim3(blocks), dim3(PB), 0, st, a);
  return hipGetLastError();
}

}  // namespace fsk
