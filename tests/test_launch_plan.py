"""Host logic: the launch plan of the staged applies (csrc/plan.h), built with the host C++
compiler and checked on seeded synthetic layouts.  The plan decides which workgroup rows a
launch has (pieces of the output tiles' stage units), their dispatch order, and the partial
slots of cut tiles; the device results of cut layouts are compared with the oracle in the
GPU parity tests."""
import json
import math
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2009_10173_amd", "csrc")

DRIVER = r"""
#include "plan.h"
#include <cstdio>
#include <iostream>
int main() {
  std::string mode;
  while (std::cin >> mode) {
    if (mode == "sim") {
      int n, patches, slots;
      std::cin >> n >> patches >> slots;
      std::vector<double> w(n);
      for (auto& x : w) std::cin >> x;
      std::printf("{\"time\": %.17g}\n", aroam::simulate_launch(w, patches, slots));
      continue;
    }
    int nT, nU, patches, slots, allow;
    double slot_bytes, max_bytes;
    std::cin >> nT;
    std::vector<int> tu(nT + 1);
    for (auto& x : tu) std::cin >> x;
    std::vector<std::vector<int>> cs(nT);
    for (auto& c : cs) {
      int k;
      std::cin >> k;
      c.resize(k);
      for (auto& x : c) std::cin >> x;
    }
    std::cin >> nU;
    std::vector<double> w(nU);
    for (auto& x : w) std::cin >> x;
    std::cin >> patches >> slots >> allow >> slot_bytes >> max_bytes;
    const aroam::LaunchPlan p =
        aroam::plan_launch(tu, cs, w, patches, slots, allow != 0, slot_bytes, max_bytes);
    std::printf("{\"pieces\": [");
    for (size_t i = 0; i < p.pieces.size(); ++i)
      std::printf("%s[%d, %d, %d, %d, %.17g]", i ? ", " : "", p.pieces[i].tile, p.pieces[i].u0,
                  p.pieces[i].u1, p.pieces[i].slot, p.pieces[i].work);
    std::printf("], \"tile_pieces\": [");
    for (int t = 0; t < nT; ++t) std::printf("%s%d", t ? ", " : "", p.tile_pieces[t]);
    std::printf("], \"tile_first_slot\": [");
    for (int t = 0; t < nT; ++t) std::printf("%s%d", t ? ", " : "", p.tile_first_slot[t]);
    std::printf("], \"n_slots\": %d, \"cut\": %d, \"heaviest_first\": %d, \"time\": %.17g, "
                "\"uncut_time\": %.17g}\n", p.n_slots, p.cut, (int)p.heaviest_first, p.time,
                p.uncut_time);
  }
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("plan")
    src = d / "plan_driver.cpp"
    src.write_text(DRIVER)
    exe = d / "plan_driver"
    subprocess.run(["g++", "-std=c++17", "-O2", "-Wall", "-Werror", "-I", CSRC, str(src), "-o",
                    str(exe)], check=True)

    def run(lines):
        out = subprocess.run([str(exe)], input="\n".join(lines) + "\n", capture_output=True,
                             text=True, check=True).stdout
        return [json.loads(x) for x in out.strip().split("\n")]
    return run


def _case_text(tile_units, chunk_starts, work, patches, slots, allow, slot_bytes=1.0,
               max_bytes=1e18):
    parts = ["plan", str(len(tile_units) - 1), " ".join(map(str, tile_units))]
    for c in chunk_starts:
        parts.append(f"{len(c)} " + " ".join(map(str, c)))
    parts.append(f"{len(work)} " + " ".join(repr(float(w)) for w in work))
    parts.append(f"{patches} {slots} {int(allow)} {slot_bytes!r} {max_bytes!r}")
    return " ".join(parts)


def _random_layout(rng):
    n_tiles = int(rng.integers(1, 13))
    sizes = rng.integers(0, 31, size=n_tiles)
    sizes[rng.random(n_tiles) < 0.15] = 0
    tile_units = [0] + list(np.cumsum(sizes).astype(int))
    chunk_starts = []
    for t in range(n_tiles):
        a, b = tile_units[t], tile_units[t + 1]
        if a == b:
            chunk_starts.append([])
            continue
        inner = [u for u in range(a + 1, b) if rng.random() < 0.35]
        chunk_starts.append([a] + inner)
    heavy = rng.random(n_tiles) < 0.3
    work = []
    for t in range(n_tiles):
        scale = 8.0 if heavy[t] else 1.0
        work += list(rng.integers(1, 20, size=sizes[t]) * scale)
    return tile_units, chunk_starts, work


def _check_plan(p, tile_units, chunk_starts, work, patches, slot_bytes, max_bytes, allow):
    n_tiles = len(tile_units) - 1
    pieces = p["pieces"]
    prefix = np.concatenate([[0.0], np.cumsum(work)])
    # each tile's units are partitioned by its pieces, cut only at chunk starts
    for t in range(n_tiles):
        mine = sorted((x for x in pieces if x[0] == t), key=lambda x: (x[1], x[2]))
        a, b = tile_units[t], tile_units[t + 1]
        assert len(mine) == p["tile_pieces"][t] >= 1
        assert mine[0][1] == a and mine[-1][2] == b
        for x, y in zip(mine, mine[1:]):
            assert x[2] == y[1] and x[1] < x[2]
        for x in mine[1:]:
            assert x[1] in chunk_starts[t]
        for x in mine:
            assert math.isclose(x[4], prefix[x[2]] - prefix[x[1]], rel_tol=1e-12, abs_tol=1e-9)
        # slots: -1 for an uncut tile, else consecutive from the tile's first slot in unit order
        if len(mine) == 1:
            assert mine[0][3] == -1 and p["tile_first_slot"][t] == -1
        else:
            first = p["tile_first_slot"][t]
            assert [x[3] for x in mine] == list(range(first, first + len(mine)))
    cut_tiles = [t for t in range(n_tiles) if p["tile_pieces"][t] > 1]
    expect_first = 0
    for t in cut_tiles:
        assert p["tile_first_slot"][t] == expect_first
        expect_first += p["tile_pieces"][t]
    assert p["n_slots"] == expect_first
    assert len(pieces) == sum(p["tile_pieces"])
    # dispatch order
    if p["heaviest_first"]:
        ws = [x[4] for x in pieces]
        assert all(u >= v for u, v in zip(ws, ws[1:]))
    else:
        assert [(x[0], x[1]) for x in pieces] == sorted((x[0], x[1]) for x in pieces)
    # a cut only where allowed, where it pays and where its slots fit
    if not allow:
        assert p["cut"] == 1 and p["n_slots"] == 0
    if p["cut"] > 1:
        assert p["time"] < 0.9 * p["uncut_time"]
        assert p["n_slots"] * patches * slot_bytes <= max_bytes
    else:
        assert p["n_slots"] == 0
    assert p["time"] <= p["uncut_time"]


def test_simulated_launch_closed_forms(driver):
    """Equal workgroups fill the places in whole rounds: n pieces x p patches of work w on s
    places take ceil(n p / s) w; one piece on more places than patches takes w."""
    cases, expect = [], []
    for n, p, s, w in [(4, 3, 5, 2.0), (7, 10, 8, 1.5), (1, 3, 8, 4.0), (3, 256, 768, 1.0),
                       (5, 200, 768, 3.0)]:
        cases.append(f"sim {n} {p} {s} " + " ".join([repr(w)] * n))
        expect.append(math.ceil(n * p / s) * w)
    # list scheduling of unequal work: two places, pieces 3, 1, 1, 1 (one patch each)
    cases.append("sim 4 1 2 3 1 1 1")
    expect.append(3.0)
    got = [r["time"] for r in driver(cases)]
    assert got == pytest.approx(expect, rel=0, abs=1e-12)


def test_random_layouts_satisfy_the_plan_invariants(driver):
    rng = np.random.default_rng(2009)
    cases, meta = [], []
    for _ in range(200):
        tu, cs, work = _random_layout(rng)
        patches = int(rng.choice([1, 3, 25, 175]))
        slots = int(rng.choice([8, 96, 768]))
        allow = bool(rng.random() < 0.7)
        slot_bytes = float(rng.choice([1.0, 16384.0]))
        max_bytes = float(rng.choice([1e18, 5e6]))
        cases.append(_case_text(tu, cs, work, patches, slots, allow, slot_bytes, max_bytes))
        meta.append((tu, cs, work, patches, slot_bytes, max_bytes, allow))
    plans = driver(cases)
    n_cut = 0
    for p, m in zip(plans, meta):
        _check_plan(p, *m)
        n_cut += p["cut"] > 1
    assert n_cut > 10  # the cut path is exercised


def test_one_heavy_tile_is_cut_and_balanced_tiles_are_not(driver):
    """A launch with far fewer workgroups than places is as long as its heaviest workgroup, so
    cutting the heavy tile pays; equal tiles over many patches fill the places evenly."""
    # tile 0: 8 units of work 10 with a chunk start every unit; tiles 1-3: 2 units of work 1
    tu = [0, 8, 10, 12, 14]
    cs = [list(range(8)), [8], [10], [12]]
    work = [10.0] * 8 + [1.0] * 6
    heavy, = driver([_case_text(tu, cs, work, patches=2, slots=64, allow=True)])
    assert heavy["cut"] > 1 and heavy["tile_pieces"][0] > 1
    assert heavy["time"] < 0.5 * heavy["uncut_time"]
    tu = [0, 4, 8, 12, 16]
    cs = [[0, 2], [4, 6], [8, 10], [12, 14]]
    work = [5.0] * 16
    even, = driver([_case_text(tu, cs, work, patches=192, slots=768, allow=True)])
    assert even["cut"] == 1 and even["n_slots"] == 0


def test_dispatch_order_is_the_one_the_simulation_finishes_sooner(driver):
    """Heaviest first is the usual winner (a heavy tile dispatched last leaves a long tail),
    but list scheduling can finish sooner in tile order: workgroups of 3, 2, 2, 3, 2 units
    (work + 1) on two places end at 6 in that order and at 7 heaviest first."""
    heavy_last, tile_wins = driver([
        _case_text([0, 1, 2, 3, 4], [[0], [1], [2], [3]], [1.0, 1.0, 1.0, 9.0], patches=3,
                   slots=4, allow=False),
        _case_text([0, 1, 2, 3, 4, 5], [[0], [1], [2], [3], [4]], [2.0, 1.0, 1.0, 2.0, 1.0],
                   patches=1, slots=2, allow=False)])
    assert heavy_last["heaviest_first"] and heavy_last["pieces"][0][0] == 3
    assert not tile_wins["heaviest_first"] and tile_wins["time"] == 6.0
    assert [x[0] for x in tile_wins["pieces"]] == [0, 1, 2, 3, 4]
