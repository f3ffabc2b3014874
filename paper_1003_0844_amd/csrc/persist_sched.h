// Host layout of the persistent grid launch (persist.hip): the order of the
// work queue, its dependency check and the packed descriptors.  Host code
// only, free of device calls, so that the scheduling can be exercised on its
// own.
#pragma once
#include <algorithm>
#include <cstring>
#include <vector>

#include "../../include/fstat.h"
#include "internal.h"

// What the schedule needs of a segment: its FFT shape and twiddle tables.
struct SegShape {
  int64_t nfft;
  int32_t R, Ceff;
  PSegTw tw;
};

inline size_t psched_align(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

struct PersistSched {
  std::vector<double> sky_ad;
  std::vector<NodeDev> ndev;
  std::vector<int32_t> node_batch;
  std::vector<PBatch> batches;
  std::vector<PUnit> units;
  std::vector<PSegTw> tw;
  size_t max_quads = 0;   // bytes per sky set
  int max_sky = 0;
  int64_t slot_elems = 0;
  int nslots = 0;
  int64_t ncnt = 0;       // 32-bit counters
  int64_t best_off = 0;   // 32-bit words from the counters to the per-node maximum keys (max mode)
  int64_t nzero = 0;      // 32-bit words the launch clears: counters and keys
  size_t desc_bytes = 0, need_ws = 0;
  bool ordered = false;   // every tile's dependencies lie earlier in the queue (checked)
};

// Whether every stage of the queue comes after the stages it waits for (the
// condition under which every wait of the persistent kernel ends).
inline bool queue_is_ordered(const PersistSched& ps) {
  const int nb = (int)ps.batches.size(), nn = (int)ps.ndev.size();
  std::vector<int64_t> sky_first(nb, -1), sky_last(nb, -1), p1_first(nn, -1), p1_last(nn, -1), p2_first(nn, -1),
      p2_last(nn, -1);
  for (int64_t u = 0; u < (int64_t)ps.units.size(); ++u) {
    const PUnit& x = ps.units[u];
    std::vector<int64_t>& f = x.kind == PU_SKY ? sky_first : (x.kind == PU_P1 ? p1_first : p2_first);
    std::vector<int64_t>& l = x.kind == PU_SKY ? sky_last : (x.kind == PU_P1 ? p1_last : p2_last);
    if (f[x.id] < 0) f[x.id] = u;
    l[x.id] = u;
  }
  for (int b = 0; b < nb; ++b) {
    if (sky_first[b] < 0) return false;
    if (b >= 2)
      for (int n = ps.batches[b - 2].node0; n < ps.batches[b - 2].node0 + ps.batches[b - 2].nnode; ++n)
        if (!(p2_last[n] >= 0 && p2_last[n] < sky_first[b])) return false;
  }
  for (int n = 0; n < nn; ++n) {
    const int b = ps.node_batch[n];
    if (p1_first[n] < 0 || p2_first[n] < 0) return false;
    if (!(sky_last[b] < p1_first[n] && p1_last[n] < p2_first[n])) return false;
    if (n >= ps.nslots && !(p2_last[n - ps.nslots] < p1_first[n])) return false;
  }
  return true;
}

// Nodes ordered by FFT length (longest first), then segment and sky position;
// batches of up to 64 sky positions of one segment; then the queue: the sky
// stage of batches 0 and 1, and for every node its pass-1 tiles followed by
// the pass-2 tiles of the node L = nslots / 2 places earlier.  The sky stage of
// batch c + 1 (whose sky set batch c - 1 used) goes in after node L + 1 of
// batch c, once every pass-2 tile of batch c - 1 is in the queue.  Every
// tile's dependencies thus lie earlier in the queue.
inline void schedule_persistent(const std::vector<SegShape>& segs, int nslots, const fstat_node* nodes, int64_t n_nodes,
                                PersistSched& ps) {
  std::vector<int64_t> order(n_nodes);
  for (int64_t i = 0; i < n_nodes; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
    const fstat_node &x = nodes[a], &y = nodes[b];
    const int64_t fa = segs[x.seg].nfft, fb = segs[y.seg].nfft;
    if (fa != fb) return fa > fb;
    if (x.seg != y.seg) return x.seg < y.seg;
    if (x.alpha != y.alpha) return x.alpha < y.alpha;
    return x.delta < y.delta;
  });
  int64_t i = 0;
  while (i < n_nodes) {
    const int sg = nodes[order[i]].seg;
    const SegShape& d = segs[sg];
    PBatch b{sg, (int)(ps.batches.size() % 2), (int)(ps.sky_ad.size() / 2), 0, (int)ps.ndev.size(), 0, 0, 0};
    while (i < n_nodes && nodes[order[i]].seg == sg) {
      const fstat_node& nd = nodes[order[i]];
      const bool new_sky = b.nsky == 0 || ps.sky_ad[ps.sky_ad.size() - 2] != nd.alpha || ps.sky_ad.back() != nd.delta;
      if (new_sky) {
        if (b.nsky == 64) break;
        ps.sky_ad.push_back(nd.alpha);
        ps.sky_ad.push_back(nd.delta);
        ++b.nsky;
      }
      ps.ndev.push_back(NodeDev{nd.fdot, (double)nd.bin_offset / (double)d.nfft, b.nsky - 1, (int32_t)order[i]});
      ps.node_batch.push_back((int32_t)ps.batches.size());
      ++b.nnode;
      ++i;
    }
    const int64_t positions = (int64_t)d.R * d.Ceff;
    b.nblk = (int)((positions + 256 * PREP_POS - 1) / (256 * PREP_POS));
    b.nprep = (b.nsky + 7) / 8 * b.nblk;
    ps.batches.push_back(b);
  }
  const int nb = (int)ps.batches.size();
  ps.nslots = nslots;
  // Pass 2 of a node L nodes after its pass 1, and pass 1 of a node nslots - L
  // nodes after pass 2 of the slot's previous user: both gaps as wide as the
  // slots allow, since a workgroup claims several tiles ahead.
  const int L = ps.nslots / 2;
  for (const auto& b : ps.batches) {
    const SegShape& d = segs[b.seg];
    ps.max_quads = std::max(ps.max_quads, (size_t)b.nsky * d.R * d.Ceff * sizeof(Quad<float>));
    ps.max_sky = std::max(ps.max_sky, b.nsky);
    ps.slot_elems = std::max(ps.slot_elems, d.nfft);
  }
  auto emit = [&](int kind, int id, int64_t tiles) {
    for (int64_t s = 0; s * PUNIT < tiles; ++s) ps.units.push_back(PUnit{kind, id, (int32_t)s, 0});
  };
  auto R_of = [&](int n) { return (int64_t)segs[ps.batches[ps.node_batch[n]].seg].R; };
  std::vector<int> pending;  // nodes whose pass 2 is not yet in the queue, oldest first
  size_t head = 0;
  auto emit_p2_through = [&](int last_batch) {  // pass 2 of every pending node of batches <= last_batch
    while (head < pending.size() && ps.node_batch[pending[head]] <= last_batch) {
      emit(PU_P2, pending[head], R_of(pending[head]));
      ++head;
    }
  };
  for (int b = 0; b < std::min(nb, 2); ++b) emit(PU_SKY, b, ps.batches[b].nprep + 2);
  for (int c = 0; c < nb; ++c) {
    const PBatch& bt = ps.batches[c];
    const int trigger = std::min(L + 1, bt.nnode - 1);
    for (int k = 0; k < bt.nnode; ++k) {
      const int n = bt.node0 + k;
      emit(PU_P1, n, R_of(n));
      pending.push_back(n);
      if ((int)(pending.size() - head) > L) {
        emit(PU_P2, pending[head], R_of(pending[head]));
        ++head;
      }
      if (k == trigger && c >= 1 && c + 1 < nb) {
        emit_p2_through(c - 1);
        emit(PU_SKY, c + 1, ps.batches[c + 1].nprep + 2);
      }
    }
  }
  emit_p2_through(nb);
  ps.ordered = queue_is_ordered(ps);
  ps.tw.resize(segs.size());
  for (size_t s = 0; s < segs.size(); ++s) ps.tw[s] = segs[s].tw;
  ps.ncnt = 4 * (int64_t)nb + 2 * (int64_t)ps.ndev.size();
  ps.best_off = (ps.ncnt + 1) / 2 * 2;
  ps.nzero = ps.best_off + 2 * (int64_t)ps.ndev.size();
  ps.desc_bytes = psched_align(ps.sky_ad.size() * sizeof(double)) + psched_align(ps.ndev.size() * sizeof(NodeDev)) +
                  psched_align(ps.node_batch.size() * sizeof(int32_t)) + psched_align(ps.batches.size() * sizeof(PBatch)) +
                  psched_align(ps.units.size() * sizeof(PUnit)) + psched_align(ps.tw.size() * sizeof(PSegTw));
  ps.need_ws = ps.desc_bytes + 2 * (psched_align(ps.max_quads) + psched_align(ps.max_sky * sizeof(SkyConst)) +
                                    psched_align(ps.max_sky * sizeof(SkyCoef))) +
               psched_align((size_t)ps.nslots * ps.slot_elems * sizeof(Pair<float>)) +
               psched_align(ps.nzero * sizeof(uint32_t)) +
               psched_align(sizeof(unsigned long long)) + 4096;
}

inline void pack_persistent(const PersistSched& ps, char* hp) {
  size_t off = 0;
  auto put = [&](const void* src, size_t bytes) {
    std::memcpy(hp + off, src, bytes);
    off += psched_align(bytes);
  };
  put(ps.sky_ad.data(), ps.sky_ad.size() * sizeof(double));
  put(ps.ndev.data(), ps.ndev.size() * sizeof(NodeDev));
  put(ps.node_batch.data(), ps.node_batch.size() * sizeof(int32_t));
  put(ps.batches.data(), ps.batches.size() * sizeof(PBatch));
  put(ps.units.data(), ps.units.size() * sizeof(PUnit));
  put(ps.tw.data(), ps.tw.size() * sizeof(PSegTw));
}

