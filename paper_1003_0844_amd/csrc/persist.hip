// The whole grid call (Sec. VI A-B: sky preparation, both FFT passes, the F
// combination and the output) in one launch of a persistent kernel.
//
// The host lays the call out as a queue of tiles (PersistArgs, internal.h):
// for every batch of sky positions its set-up, record and coefficient tiles,
// for every node its R first-pass tiles and its R second-pass tiles, in an
// order where every tile depends only on tiles before it.  A workgroup claims
// `chunk` consecutive tiles at a time from a global counter (a chunk never
// crosses a unit of PUNIT tiles, so the tiles of a pass-1 or pass-2 chunk
// belong to one node), and for each tile waits until what the tile reads is
// complete, runs it with the same tile functions as the launch-per-pass
// kernels (tiles.h), and counts it complete.
//
// Dependencies (completion counters, cnt):
//   set-up of batch b      after batch b-2 (same sky set) has finished pass 2
//   record / coefficient   after the set-up of b
//   pass 1 of node n       after all record tiles of its batch, and after
//                          pass 2 of node n - nslots (the spill slot's last user)
//   pass 2 of node n       after pass 1 of n and the coefficients of its batch
// Completion is published with an agent-scope release (writer) and observed
// with an agent-scope acquire (reader): the workgroups of one dependency run
// on different XCDs, whose L2 caches are not coherent with each other.  Both
// act on a whole L2, so a workgroup pays for them once per run of tiles, not
// per tile: completions of tiles that count on the same counters are added up
// (Pending) and published when the counter changes, before the workgroup
// waits on a counter it has completions pending on, before it claims the next
// chunk, and when it leaves; a wait already seen satisfied by the workgroup
// (Seen) is not repeated (counters only grow, and every counter belongs to one
// batch or node of the call, whose data do not change once complete).
//
// Every wait ends: by induction over the queue, the earliest tile not yet
// complete has all its dependencies earlier in the queue, claimed by running
// workgroups (a workgroup claims only while it runs) and complete; their
// completions are published at the latest when their workgroups claim again
// or leave, or before those workgroups wait on them.  Each wait is also bounded
// in wall-clock time: past spin_ticks it sets the sticky error flag and every
// workgroup leaves the queue, so the kernel ends in any case.
//
// Max mode needs no partials read across XCDs: a workgroup keeps the
// largest F of its run of pass-2 tiles of a node as an ordered (F, bin) key,
// takes an atomic maximum of it into the node's key when it publishes the
// run, and the workgroup whose publication completes the node's pass 2
// writes the output.
//
// Pass 2 of node n interleaves with pass 1 of node n + L in the queue (L =
// nslots / 2, chosen by the host), so at most nslots nodes' spill is live.
#include "tiles.h"

namespace {

constexpr int PB = 256;   // threads per workgroup
constexpr int PC = 4096;  // first-pass length
constexpr int P_LDS = lds_slots(PC, 1);
static_assert(lds_slots(256, 16) == P_LDS && lds_slots(64, 64) == P_LDS && lds_slots(1024, 4) == P_LDS,
              "second-pass tiles with R x B2 = 4096 use the first pass's LDS");

// counters: per batch b at 4 b: set-up, record tiles, coefficients, pass-2
// tiles; per node n at 4 nbatch + 2 n: pass-1 tiles, pass-2 tiles
__device__ __forceinline__ uint32_t* batch_cnt(const PersistArgs& a, int b, int which) { return a.cnt + 4 * b + which; }
__device__ __forceinline__ uint32_t* node_cnt(const PersistArgs& a, int n, int which) {
  return a.cnt + 4 * (int64_t)a.nbatch + 2 * (int64_t)n + which;
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

// Everything the workgroup wrote before the barrier that precedes this (one
// thread) becomes visible to agent-scope acquirers of what it counts next.
// The explicit wait after the fence keeps the L2 write-back complete before
// the count: at the head of the claim loop, with the previous tile's stores
// still in flight on the back edge, the compiler omits the wait the fence
// implies.
__device__ __forceinline__ void release_agent() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __builtin_amdgcn_s_waitcnt(0);
}

__device__ __forceinline__ void acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

// Max mode: (F, k) as a key whose unsigned order is that of F, then of the
// lower bin (0 <= k < 2^32).  -0 counts as +0, as in the comparison of the
// launch-per-pass reduction.
__device__ __forceinline__ unsigned long long max_key(float F, int64_t k) {
  uint32_t u = __float_as_uint(F == 0.0f ? 0.0f : F);
  u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
  return ((unsigned long long)u << 32) | (unsigned long long)(0xFFFFFFFFu - (uint32_t)k);
}
__device__ __forceinline__ void max_unkey(unsigned long long key, float& F, int64_t& k) {
  if (key == 0ull) {  // no bin in [k_lo, k_hi): as the launch-per-pass reduction leaves it
    F = -1.0f;
    k = INT64_MAX;
    return;
  }
  uint32_t u = (uint32_t)(key >> 32);
  u = (u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u;
  F = __uint_as_float(u);
  k = (int64_t)(0xFFFFFFFFu - (uint32_t)key);
}

// Completions thread 0 has counted but not yet published: n tiles on c
// and, if c2 is set, on c2 (a count that only orders the reuse of a sky set).
// Max mode: node >= 0 for pass-2 tiles, key their largest (F, bin), R the
// node's tile count.
struct Pending {
  uint32_t* c = nullptr;
  uint32_t* c2 = nullptr;
  uint32_t n = 0;
  int32_t node = -1, R = 0;
  unsigned long long key = 0ull;
};

template <int MODE>
__device__ __forceinline__ void publish(const PersistArgs& a, Pending& p) {
  if (p.n) {
    const bool mx = MODE == 1 && p.node >= 0;
    if (mx && p.key) {
      __hip_atomic_fetch_max(a.best + p.node, p.key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_s_waitcnt(0);  // the maximum is in place before the tiles count
    }
    release_agent();
    const uint32_t old = __hip_atomic_fetch_add(p.c, p.n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (p.c2) __hip_atomic_fetch_add(p.c2, p.n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (mx && old + p.n == (uint32_t)p.R) {  // the node's last pass-2 tiles: its output
      float F;
      int64_t k;
      max_unkey(__hip_atomic_load(a.best + p.node, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), F, k);
      const int row = a.nodes[p.node].row;
      ((float*)a.out.Fmax)[row] = F;
      a.out.kmax[row] = k;
    }
  }
  p.n = 0;
  p.key = 0ull;
}

// Count the tile about to run (published only after the barrier that ends it).
template <int MODE>
__device__ __forceinline__ void count(const PersistArgs& a, Pending& p, uint32_t* c, uint32_t* c2, int node = -1,
                                      int R = 0) {
  if (p.n && (p.c != c || p.c2 != c2)) publish<MODE>(a, p);
  p.c = c;
  p.c2 = c2;
  p.node = node;
  p.R = R;
  ++p.n;
}

// The last two waits thread 0 found satisfied.
struct Seen {
  const uint32_t* c[2] = {nullptr, nullptr};
  uint32_t t[2] = {0u, 0u};
};

// Thread 0: make sure *c >= t before the tile runs.  A wait seen satisfied
// before is not repeated; completions pending on c are published first (the
// tile may need them); `waited` records that an acquire must follow.
template <int MODE>
__device__ bool need(const PersistArgs& a, Pending& p, Seen& s, bool& waited, const uint32_t* c, uint32_t t) {
  if ((s.c[0] == c && s.t[0] >= t) || (s.c[1] == c && s.t[1] >= t)) return true;
  if (p.n && (p.c == c || p.c2 == c)) publish<MODE>(a, p);
  if (!wait_ge(a, c, t)) return false;
  s.c[1] = s.c[0];
  s.t[1] = s.t[0];
  s.c[0] = c;
  s.t[0] = t;
  waited = true;
  return true;
}

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
__device__ __forceinline__ MaxPartial pass2_of(const SegDev& sg, const PersistArgs& a, const PSegTw& tw,
                                               const PBatch& bt, int n, int cb, lds_t<Pair<float>>* lds) {
  const NodeDev node = a.nodes[n];
  const int slot = n % a.nslots;
  return pass2_tile<float, R, MODE>(sg, (const Pair<float>*)a.spill + (int64_t)slot * a.slot_elems, node,
                                    a.coef[bt.set][node.sky], (const cpx<float>*)tw.twR, a.out, cb, nullptr, lds);
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
  __shared__ int s_ok;
  const int tid = threadIdx.x;
  // Control flow: every branch that decides which barrier a thread reaches
  // next is taken on a wave-uniform value (the claimed item, or a flag thread
  // 0 left in LDS, read with readfirstlane), and every thread-0 block is
  // followed by a barrier before such a branch.  With a thread-0 block in
  // front of the loop latch and another behind it, the compiler may merge the
  // two tests of tid == 0 and send threads 1.. straight back to the barrier
  // after the claim while thread 0's lane waits outside that inner loop: the
  // workgroup would run the same tile over and over and never claim another.
  // So thread 0 does its bookkeeping in the block before each tile (and in the
  // claim block), and every tile ends with a barrier.
  Pending pd;                // thread 0
  Seen seen;                 // thread 0
  int64_t nxt = 0, lim = 0;  // thread 0: the claimed range of items
  for (;;) {
    if (tid == 0) {
      if (nxt >= lim) {
        publish<MODE>(a, pd);
        nxt = (int64_t)atomicAdd(a.head, (unsigned long long)a.chunk);
        lim = nxt + a.chunk;
      }
      s_item = (unsigned long long)nxt++;
    }
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
        bool waited = false, ok;
        if (tile == 0) {
          ok = b < 2 || need<MODE>(a, pd, seen, waited, batch_cnt(a, b - 2, 3),
                             (uint32_t)(a.batches[b - 2].nnode * a.segs[a.batches[b - 2].seg].R));
        } else {
          ok = need<MODE>(a, pd, seen, waited, batch_cnt(a, b, 0), 1u);
        }
        if (ok) {
          if (waited) acquire();
          count<MODE>(a, pd, batch_cnt(a, b, tile == 0 ? 0 : (tile <= bt.nprep ? 1 : 2)), nullptr);
        }
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
        bool waited = false;
        bool ok = need<MODE>(a, pd, seen, waited, batch_cnt(a, b, 1), (uint32_t)bt.nprep);
        if (ok && n >= a.nslots) {
          const int m = n - a.nslots;
          ok = need<MODE>(a, pd, seen, waited, node_cnt(a, m, 1), (uint32_t)a.segs[a.batches[a.node_batch[m]].seg].R);
        }
        if (ok) {
          if (waited) acquire();
          count<MODE>(a, pd, node_cnt(a, n, 0), nullptr);
        }
        s_ok = ok;
      }
      __syncthreads();
      if (!uniform_flag(s_ok)) break;
      if (R > 128) pass1_of<true>(sg, a, tw, bt, n, tile, lds);  // the spill layout of pass 2's B2
      else pass1_of<false>(sg, a, tw, bt, n, tile, lds);
      __syncthreads();
      continue;
    }

    // pass 2, column block `tile` of node n
    if (tid == 0) {
      bool waited = false;
      bool ok = need<MODE>(a, pd, seen, waited, node_cnt(a, n, 0), (uint32_t)R);
      if (ok) ok = need<MODE>(a, pd, seen, waited, batch_cnt(a, b, 2), 1u);
      if (ok) {
        if (waited) acquire();
        count<MODE>(a, pd, node_cnt(a, n, 1), batch_cnt(a, b, 3), n, R);
      }
      s_ok = ok;
    }
    __syncthreads();
    if (!uniform_flag(s_ok)) break;
    MaxPartial mx;
    switch (R) {
      case 64: mx = pass2_of<64, MODE>(sg, a, tw, bt, n, tile, lds); break;
      case 128: mx = pass2_of<128, MODE>(sg, a, tw, bt, n, tile, lds); break;
      case 256: mx = pass2_of<256, MODE>(sg, a, tw, bt, n, tile, lds); break;
      case 512: mx = pass2_of<512, MODE>(sg, a, tw, bt, n, tile, lds); break;
      default: mx = pass2_of<1024, MODE>(sg, a, tw, bt, n, tile, lds); break;
    }
    if constexpr (MODE == 1) {
      // the block's maximum joins the run's key (thread 0 holds both)
      if (tid == 0 && mx.k != INT64_MAX) {
        const unsigned long long key = max_key((float)mx.F, mx.k);
        if (key > pd.key) pd.key = key;
      }
    }
    __syncthreads();
  }
  // completions still pending (the loop ends at a claim past the queue, or on an error)
  if (tid == 0) publish<MODE>(a, pd);
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
  if (blocks <= 0 || a.chunk <= 0 || PUNIT % a.chunk != 0) return hipErrorInvalidValue;
  if (mode == 0) hipLaunchKernelGGL(k_persist<0>, dim3(blocks), dim3(PB), 0, st, a);
  else if (mode == 1) hipLaunchKernelGGL(k_persist<1>, dim3(blocks), dim3(PB), 0, st, a);
  else hipLaunchKernelGGL(k_persist<2>, dim3(blocks), dim3(PB), 0, st, a);
  return hipGetLastError();
}

}  // namespace fsk
