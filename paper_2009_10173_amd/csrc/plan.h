// Launch plan of a staged apply: which workgroup rows the launch has, in which order they are
// dispatched, and which tiles are cut into pieces (host code only, no device types, so that
// it can be built and tested on its own).
//
// A staged launch has one workgroup per (piece, position patch).  A piece is a range of one
// output tile's stage units.  An uncut tile is one piece, which writes the output; a cut
// tile is several pieces, cut where a chunk starts (the LDS ring is reloaded there anyway),
// and each of them writes its partial sums to its own slot, which a second kernel adds in
// slot order.  The slots of a tile are consecutive and follow the tile's unit order, so the
// sum is deterministic.
#pragma once

#include <algorithm>
#include <cmath>
#include <functional>
#include <queue>
#include <vector>

namespace aroam {

struct PlanPiece {
  int tile, u0, u1;  // units [u0, u1) of the tile
  int slot;          // partial slot, or -1 for the single piece of an uncut tile
  double work;
};

struct LaunchPlan {
  std::vector<PlanPiece> pieces;     // in dispatch order
  std::vector<int> tile_pieces;      // [tile] pieces of the tile
  std::vector<int> tile_first_slot;  // [tile] slot of its first piece, -1 when uncut
  int n_slots = 0;
  int cut = 1;                       // D of the chosen cut (1: no tile cut)
  bool heaviest_first = false;
  double time = 0;                   // simulated finishing time (work units)
  double uncut_time = 0;             // the same without cuts
};

// Finishing time of a launch whose workgroups (every patch of each piece, pieces in the given
// order) take the first of `slots` free places and last as long as their work.
inline double simulate_launch(const std::vector<double>& piece_work, int n_patches, int slots) {
  std::priority_queue<double, std::vector<double>, std::greater<double>> free_at;
  for (int i = 0; i < slots; ++i) free_at.push(0.0);
  double end = 0;
  for (double w : piece_work)
    for (int p = 0; p < n_patches; ++p) {
      const double t = free_at.top() + w;
      free_at.pop();
      free_at.push(t);
      end = std::max(end, t);
    }
  return end;
}

// Plan a launch.  tile_units[t] .. tile_units[t + 1] are tile t's units; chunk_starts[t]
// lists the units of tile t where a chunk starts (the first is tile_units[t] when the tile
// has units); unit_work[u] is unit u's work.  For D = 1 .. 8 every tile is cut into about
// (its work) / (largest tile work / D) pieces of similar work, each cut at the chunk start
// whose prefix work is nearest to its share, and the pieces are dispatched in tile order or
// heaviest first, whichever the simulation (`slots` places, one workgroup per piece and
// patch, one unit of work added per workgroup for its fixed costs) finishes sooner.  A cut
// is taken only when `allow_cut`, when it shortens the simulated launch by more than 10 %,
// and when its slots (slot_bytes per piece and patch) fit in max_slot_bytes.
inline LaunchPlan plan_launch(const std::vector<int>& tile_units,
                              const std::vector<std::vector<int>>& chunk_starts,
                              const std::vector<double>& unit_work, int n_patches, int slots,
                              bool allow_cut, double slot_bytes, double max_slot_bytes) {
  const int nT = (int)tile_units.size() - 1;
  std::vector<double> prefix(unit_work.size() + 1, 0.0);
  for (size_t u = 0; u < unit_work.size(); ++u) prefix[u + 1] = prefix[u] + unit_work[u];
  double wmax = 0;
  for (int t = 0; t < nT; ++t)
    wmax = std::max(wmax, prefix[tile_units[t + 1]] - prefix[tile_units[t]]);
  auto cut = [&](int D, std::vector<PlanPiece>& out, std::vector<int>& npieces) {
    out.clear();
    npieces.assign(nT, 1);
    for (int t = 0; t < nT; ++t) {
      const int a = tile_units[t], b = tile_units[t + 1];
      const double wt = prefix[b] - prefix[a];
      const std::vector<int>& cs = chunk_starts[t];
      int S = 1;
      if (D > 1 && wt > 0 && wmax > 0)
        S = std::max(1, std::min((int)cs.size(), (int)std::lround(wt * D / wmax)));
      std::vector<int> cuts;
      size_t j = 1;
      for (int k = 1; k < S && j < cs.size(); ++k, ++j) {
        const double goal = prefix[a] + wt * k / S;
        while (j + 1 < cs.size() &&
               std::fabs(prefix[cs[j + 1]] - goal) <= std::fabs(prefix[cs[j]] - goal))
          ++j;
        cuts.push_back(cs[j]);
      }
      cuts.push_back(b);
      int u = a;
      for (int v : cuts) {
        out.push_back(PlanPiece{t, u, v, -1, prefix[v] - prefix[u]});
        u = v;
      }
      npieces[t] = (int)cuts.size();  // a tile without units keeps one piece that writes zeros
    }
  };
  auto launch_time = [&](const std::vector<PlanPiece>& order) {
    std::vector<double> w;
    for (const PlanPiece& p : order) w.push_back(p.work + 1.0);
    return simulate_launch(w, n_patches, slots);
  };
  LaunchPlan best;
  std::vector<PlanPiece> cur;
  std::vector<int> cur_np;
  for (int D = 1; D <= (allow_cut ? 8 : 1); ++D) {
    cut(D, cur, cur_np);
    long long nslots = 0;
    for (int t = 0; t < nT; ++t) nslots += cur_np[t] > 1 ? cur_np[t] : 0;
    if (D > 1 && (double)nslots * n_patches * slot_bytes > max_slot_bytes) break;
    std::vector<PlanPiece> heavy = cur;
    std::stable_sort(heavy.begin(), heavy.end(),
                     [](const PlanPiece& x, const PlanPiece& y) { return x.work > y.work; });
    double time = launch_time(cur);
    const double time_heavy = launch_time(heavy);
    const bool hf = time_heavy <= time;
    if (hf) {
      time = time_heavy;
      cur.swap(heavy);
    }
    if (D == 1) best.uncut_time = time;
    if (D == 1 || (time < 0.9 * best.uncut_time && time < best.time)) {
      best.pieces = cur;
      best.tile_pieces = cur_np;
      best.cut = D;
      best.heaviest_first = hf;
      best.time = time;
    }
  }
  // slots: consecutive per cut tile, in unit order
  best.tile_first_slot.assign(nT, -1);
  best.n_slots = 0;
  for (int t = 0; t < nT; ++t)
    if (best.tile_pieces[t] > 1) {
      best.tile_first_slot[t] = best.n_slots;
      best.n_slots += best.tile_pieces[t];
    }
  std::vector<int> order(best.pieces.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    return best.pieces[x].u0 < best.pieces[y].u0;
  });
  std::vector<int> seen(nT, 0);
  for (int i : order) {
    PlanPiece& p = best.pieces[i];
    if (best.tile_pieces[p.tile] > 1) p.slot = best.tile_first_slot[p.tile] + seen[p.tile]++;
  }
  return best;
}

}  // namespace aroam
