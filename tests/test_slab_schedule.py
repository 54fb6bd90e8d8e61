"""The slab-skewed chain schedule (a matrix-powers style order, Section VII) on
the CPU: the library's own ppn::slab_order (host_numerics.cpp, built here with
AddressSanitizer and UndefinedBehaviorSanitizer) replayed over per-tile buffer
versions for the three chains the library runs in that order.

For every part (launch k over tiles [t0, t1)) the replay checks that each
gathered read (tiles within the bandwidth w of the part) and each elementwise
read (the part's own tiles) sees the buffer version the full-range order gives
that launch, then applies the part's writes.  It also checks that every launch
covers every tile exactly once.  The launch lists mirror the solver's:
  * operator form (run_op_chain): real root p' = p - A p/theta, pairs as a
    product into Tb then p' = p - c1 t + c2 A t, ping-pong buffers, the last
    launch reading v elementwise and writing the output;
  * product form (run_chain, pp_apply and the cycle-end update): y accumulated
    in place, the last real root folded into the previous launch;
  * Horner (run_horner, the power basis): z <- A z + c v with v elementwise.
"""
import os
import random
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1907_00072_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <vector>
#include "host_numerics.h"
// stdin: number of cases, then per case: ntile S w K group
// stdout per case: number of parts, then "k t0 t1" per part
int main() {
  int ncase = 0;
  if (scanf("%d", &ncase) != 1) return 2;
  std::vector<ppn::SlabPart> out;
  for (int c = 0; c < ncase; ++c) {
    int ntile, S, w, K, group;
    if (scanf("%d %d %d %d %d", &ntile, &S, &w, &K, &group) != 5) return 2;
    ppn::slab_order(ntile, S, w, K, group, out);
    printf("%zu\n", out.size());
    for (const ppn::SlabPart &p : out) printf("%d %d %d\n", p.k, p.t0, p.t1);
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def order_tool(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("slab")
    drv = d / "driver.cpp"
    drv.write_text(DRIVER)
    exe = d / "driver"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-I" + CSRC,
           "-I" + os.path.join(ROOT, "include"), os.path.join(CSRC, "host_numerics.cpp"),
           str(drv), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]

    def orders(cases):
        text = f"{len(cases)}\n" + "".join(f"{a} {b} {c} {k} {g}\n" for a, b, c, k, g in cases)
        r = subprocess.run([str(exe)], input=text, capture_output=True, text=True,
                           env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
        assert r.returncode == 0, r.stderr[-2000:]
        assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
        tok = iter(r.stdout.split())
        res = []
        for _ in cases:
            m = int(next(tok))
            res.append([(int(next(tok)), int(next(tok)), int(next(tok))) for _ in range(m)])
        return res
    return orders


# ---- launch lists (gathered reads, elementwise reads, writes) of the three chains
def op_form(kinds):
    L, cur, bufs, pb = [], "v", ["P0", "P1"], 0
    for k, kind in enumerate(kinds):
        last = k == len(kinds) - 1
        dst = "out" if last else bufs[pb]
        if kind == "r":
            L.append(dict(gather=[cur], own=["v"] if last else [], write=[dst]))
        else:
            L.append(dict(gather=[cur], own=[], write=["Tb"]))
            L.append(dict(gather=["Tb"], own=[cur] + (["v"] if last else []), write=[dst]))
        cur, pb = dst, pb ^ 1
    return L


def product_form(kinds, y_in):
    L, cur, bufs, pb, yi = [], "v", ["P0", "P1"], 0, y_in
    K = len(kinds)
    for k, kind in enumerate(kinds):
        last = k == K - 1
        fold = k + 2 == K and kinds[k + 1] == "r"
        own_y = [yi] if yi else []
        if kind == "r":
            assert not last  # a single real root is an axpy, not a chain launch
            L.append(dict(gather=[cur], own=own_y, write=["y"] + ([] if fold else [bufs[pb]])))
            yi = "y"
            if fold:
                break
        else:
            L.append(dict(gather=[cur], own=own_y, write=["y"] + ([] if last else ["Tb"])))
            yi = "y"
            if last:
                break
            L.append(dict(gather=["Tb"], own=[cur, "y"],
                          write=["y"] + ([] if fold else [bufs[pb]])))
            if fold:
                break
        cur, pb = bufs[pb], pb ^ 1
    return L


def horner(deg):
    L, z, bufs, pb = [], "v", ["P0", "P1"], 0
    for k in range(deg - 1, -1, -1):
        dst = "out" if k == 0 else bufs[pb]
        L.append(dict(gather=[z], own=["v"], write=[dst]))
        z, pb = dst, pb ^ 1
    return L


def replay(L, parts, ntile, w):
    # the version each launch must read: the last earlier writer in launch order
    prod, expect = {}, []
    for i, l in enumerate(L):
        expect.append({b: prod.get(b, -1) for b in l["gather"] + l["own"]})
        for b in l["write"]:
            prod[b] = i
    names = {b for l in L for b in l["gather"] + l["own"] + l["write"]}
    ver = {b: [-1] * ntile for b in names}
    cover = [[0] * ntile for _ in L]
    for k, t0, t1 in parts:
        assert 0 <= k < len(L) and 0 <= t0 < t1 <= ntile, (k, t0, t1)
        l, e = L[k], expect[k]
        for b in l["gather"]:
            for t in range(max(0, t0 - w), min(ntile, t1 + w)):
                assert ver[b][t] == e[b], ("gather", k, b, t, ver[b][t], e[b])
        for b in l["own"]:
            for t in range(t0, t1):
                assert ver[b][t] == e[b], ("own", k, b, t, ver[b][t], e[b])
        for b in l["write"]:
            for t in range(t0, t1):
                ver[b][t] = k
        for t in range(t0, t1):
            cover[k][t] += 1
    assert all(c == 1 for row in cover for c in row)


def _cases(rng, count):
    out = []
    for _ in range(count):
        ntile = rng.choice([1, 2, 5, 17, 40, 64])
        out.append((ntile, rng.choice([1, 2, 3, 8, 20, 100]), rng.choice([0, 1, 2, 5]),
                    rng.randint(1, 24), rng.choice([1, 2, 3, 4, 8, 50, 1 << 20])))
    return out


def test_operator_form_chain(order_tool):
    rng = random.Random(11)
    chains = []
    for _ in range(500):
        kinds = [rng.choice("rp") for _ in range(rng.randint(1, 10))]
        chains.append(op_form(kinds))
    cases = [(nt, S, w, len(L), g)
             for L, (nt, S, w, _, g) in zip(chains, _cases(rng, len(chains)))]
    for L, (nt, S, w, K, g), parts in zip(chains, cases, order_tool(cases)):
        replay(L, parts, nt, w)


def test_product_form_chain(order_tool):
    rng = random.Random(12)
    chains = []
    while len(chains) < 500:
        kinds = [rng.choice("rp") for _ in range(rng.randint(2, 10))]
        chains.append(product_form(kinds, rng.choice([None, "x_in", "y"])))
    cases = [(nt, S, w, len(L), g)
             for L, (nt, S, w, _, g) in zip(chains, _cases(rng, len(chains)))]
    for L, (nt, S, w, K, g), parts in zip(chains, cases, order_tool(cases)):
        replay(L, parts, nt, w)


def test_horner_chain(order_tool):
    rng = random.Random(13)
    chains = [horner(rng.randint(1, 16)) for _ in range(300)]
    cases = [(nt, S, w, len(L), g)
             for L, (nt, S, w, _, g) in zip(chains, _cases(rng, len(chains)))]
    for L, (nt, S, w, K, g), parts in zip(chains, cases, order_tool(cases)):
        replay(L, parts, nt, w)


def test_order_shape(order_tool):
    # one group, S = 3 tiles, w = 1: launch k trails launch k-1 by one tile
    parts = order_tool([(7, 3, 1, 3, 8)])[0]
    assert parts[:5] == [(0, 0, 3), (1, 0, 2), (2, 0, 1), (0, 3, 6), (1, 2, 5)]
    # group 1 is the full-range order
    assert order_tool([(7, 100, 2, 3, 1)])[0] == [(0, 0, 7), (1, 0, 7), (2, 0, 7)]
    # edge cases: no launch; one tile; a diagonal matrix (w = 0: slabs are not skewed)
    none, one, diag = order_tool([(5, 2, 1, 0, 4), (1, 1, 0, 2, 8), (4, 2, 0, 2, 8)])
    assert none == [] and one == [(0, 0, 1), (1, 0, 1)]
    assert diag == [(0, 0, 2), (1, 0, 2), (0, 2, 4), (1, 2, 4)]


def test_a_planted_schedule_error_is_caught(order_tool):
    # the replay must reject an order whose second launch runs ahead of its input
    L = op_form("rrr")
    parts = order_tool([(10, 2, 1, len(L), 8)])[0]
    bad = sorted(parts, key=lambda p: (p[0] != 1, p))  # launch 1 first
    with pytest.raises(AssertionError):
        replay(L, bad, 10, 1)
