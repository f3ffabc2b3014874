// CPU emulation of the persistent grid kernel's control flow over the
// library's own schedule (persist_sched.h): W threads claim tiles from a
// shared counter, wait on the same completion counters with the same
// targets as the kernel, and count completion; tile bodies only record that
// they ran, after a random pause now and then, so that workgroups overtake
// each other.  Exit status 0 iff every tile ran exactly once and no wait
// outlived 5 s.  Arguments: threads, spill slots, tiles per claim.
#include <atomic>
#include <functional>
#include <chrono>
#include <cstdio>
#include <random>
#include <thread>
#include <vector>
#include "persist_sched.h"

int main(int argc, char** argv) {
  const int W = argc > 1 ? atoi(argv[1]) : 64;
  const int slots = argc > 2 ? atoi(argv[2]) : 8;
  const int chunk = argc > 3 ? atoi(argv[3]) : 1;
  std::vector<SegShape> segs = {{1 << 18, 64, 2693, {}}, {1 << 19, 128, 1347, {}}, {1 << 20, 256, 1347, {}}};
  std::mt19937 g(5);
  std::uniform_real_distribution<double> U(0, 6.28);
  std::vector<fstat_node> nodes;
  double a0 = U(g);
  nodes.push_back({a0, 0.1, -1e-10, 0, 0.f});
  for (int s = 0; s < 3; ++s) { double a = U(g); for (int f = 0; f < 2; ++f) nodes.push_back({a, 0.2, -3e-10 * f, 0, 0.f}); }
  for (int s = 0; s < 70; ++s) nodes.push_back({U(g), 0.3, -5e-10, 1, 0.f});
  for (int s = 0; s < 2; ++s) { double a = U(g); for (int f = 0; f < 3; ++f) nodes.push_back({a, 0.4, -4e-10 * f, 2, 0.f}); }
  std::shuffle(nodes.begin(), nodes.end(), g);
  PersistSched ps;
  schedule_persistent(segs, slots, nodes.data(), (int64_t)nodes.size(), ps);
  printf("nodes %zu batches %zu units %zu ordered %d\n", ps.ndev.size(), ps.batches.size(), ps.units.size(), (int)ps.ordered);
  for (auto& b : ps.batches) printf("  batch seg %d set %d nsky %d nnode %d nblk %d nprep %d\n", b.seg, b.set, b.nsky, b.nnode, b.nblk, b.nprep);
  const int nb = ps.batches.size(), nn = ps.ndev.size();
  std::vector<std::atomic<uint32_t>> cnt(4 * nb + 2 * nn);
  for (auto& c : cnt) c = 0;
  std::atomic<uint64_t> head{0};
  std::atomic<int> error{0};
  const int64_t nitems = (int64_t)ps.units.size() * PUNIT;
  std::vector<std::atomic<int>> done(nitems);
  for (auto& d : done) d = 0;
  auto bc = [&](int b, int w) -> std::atomic<uint32_t>& { return cnt[4 * b + w]; };
  auto ncn = [&](int n, int w) -> std::atomic<uint32_t>& { return cnt[4 * nb + 2 * n + w]; };
  auto R = [&](int n) { return segs[ps.batches[ps.node_batch[n]].seg].R; };
  auto wait = [&](std::atomic<uint32_t>& c, uint32_t t) {
    auto t0 = std::chrono::steady_clock::now();
    while (c.load() < t) {
      if (error.load()) return false;
      if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(5)) { error = 1; return false; }
      std::this_thread::yield();
    }
    return true;
  };
  std::atomic<int64_t> bad{0};
  // The kernel's thread-0 logic: chunked claims, completions counted before a
  // tile and published on a counter change, before a wait on a pending
  // counter, before the next claim and at the end; waits seen satisfied are
  // not repeated.
  auto worker = [&]() {
    struct Pending { std::atomic<uint32_t>* c = nullptr; std::atomic<uint32_t>* c2 = nullptr; uint32_t n = 0; } pd;
    struct Seen { std::atomic<uint32_t>* c[2] = {nullptr, nullptr}; uint32_t t[2] = {0, 0}; } seen;
    auto publish = [&]() {
      if (pd.n) {
        pd.c->fetch_add(pd.n);
        if (pd.c2) pd.c2->fetch_add(pd.n);
      }
      pd.n = 0;
    };
    auto count = [&](std::atomic<uint32_t>* c, std::atomic<uint32_t>* c2) {
      if (pd.n && (pd.c != c || pd.c2 != c2)) publish();
      pd.c = c;
      pd.c2 = c2;
      ++pd.n;
    };
    auto need = [&](std::atomic<uint32_t>& c, uint32_t t) {
      if ((seen.c[0] == &c && seen.t[0] >= t) || (seen.c[1] == &c && seen.t[1] >= t)) return true;
      if (pd.n && (pd.c == &c || pd.c2 == &c)) publish();
      if (!wait(c, t)) return false;
      seen.c[1] = seen.c[0];
      seen.t[1] = seen.t[0];
      seen.c[0] = &c;
      seen.t[0] = t;
      return true;
    };
    std::mt19937 rng(std::hash<std::thread::id>{}(std::this_thread::get_id()));
    auto pause = [&]() {
      if ((rng() & 7u) == 0)
        for (int k = (int)(rng() % 64); k > 0; --k) std::this_thread::yield();
    };
    int64_t nxt = 0, lim = 0;
    for (;;) {
      if (nxt >= lim) {
        publish();
        nxt = (int64_t)head.fetch_add(chunk);
        lim = nxt + chunk;
      }
      const int64_t item = nxt++;
      if (item >= nitems) break;
      const PUnit u = ps.units[item / PUNIT];
      const int tile = u.sub * PUNIT + (int)(item % PUNIT);
      if (u.kind == PU_SKY) {
        const int b = u.id;
        const PBatch& bt = ps.batches[b];
        if (tile >= bt.nprep + 2) { done[item] = 1; continue; }
        bool ok = tile == 0 ? (b < 2 || need(bc(b - 2, 3), ps.batches[b - 2].nnode * segs[ps.batches[b - 2].seg].R))
                            : need(bc(b, 0), 1);
        if (!ok) break;
        count(&bc(b, tile == 0 ? 0 : (tile <= bt.nprep ? 1 : 2)), nullptr);
        pause();
        done[item]++;
        continue;
      }
      const int n = u.id, b = ps.node_batch[n];
      const PBatch& bt = ps.batches[b];
      if (u.kind == PU_P1) {
        bool ok = need(bc(b, 1), bt.nprep);
        if (ok && n >= slots) ok = need(ncn(n - slots, 1), R(n - slots));
        if (!ok) break;
        count(&ncn(n, 0), nullptr);
        if (tile >= R(n)) bad++;
        pause();
        done[item]++;
        continue;
      }
      bool ok = need(ncn(n, 0), R(n));
      if (ok) ok = need(bc(b, 2), 1);
      if (!ok) break;
      count(&ncn(n, 1), &bc(b, 3));
      if (tile >= R(n)) bad++;
      pause();
      done[item]++;
    }
    publish();
  };
  std::vector<std::thread> th;
  for (int w = 0; w < W; ++w) th.emplace_back(worker);
  for (auto& t : th) t.join();
  int64_t twice = 0, never = 0;
  for (int64_t i = 0; i < nitems; ++i) { twice += done[i] > 1; never += done[i] == 0; }
  printf("W %d slots %d chunk %d: error %d, items never run %lld, run twice %lld, bad tiles %lld\n", W, slots, chunk, error.load(),
         (long long)never, (long long)twice, (long long)bad.load());
  return error.load();
}
