"""Pins of the restoration oracle (static and dynamic restoration, Sec.
"Heuristic complements", subsections "Static restoration (SR)" and
"Dynamic restoration (DR)").

The paper prints no numbers for these procedures, so the oracle is pinned by
what its definitions fix:
* special cases that reduce to the plain diffusion (eps = 0: sigma = 1;
  one interval: no mesh point to mix at), which is itself pinned against
  dense real-space matrix exponentials and closed forms;
* the defining property of the mix: on good pixels the orientation maximum
  becomes eps h0 + (1 - eps) h, with one factor for all orientations, and
  nothing changes on bad pixels;
* invariances the definitions respect (degree-1 homogeneity, 90-degree
  rotation with the orientation shift N/4);
* the DR growth rule on small hand-worked grids.
"""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from oracle import restore_oracle as RO  # noqa: E402
from paper_1304_2062_amd import synth  # noqa: E402

GOLDEN = os.path.join(ROOT, "tests", "golden")


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _case(M=32, N=16, seed=3, rho=0.4):
    f = 0.1 + 0.9 * synth.make_image(seed, M, "small")
    mask = synth.mask_random(seed + 1, M, rho) | synth.mask_stripes(M, 2, 11)
    rmap, _ = O.orient(f, mask, N)
    return f, mask, rmap


@pytest.mark.parametrize("dynamic", [False, True])
def test_eps_zero_is_the_plain_diffusion(dynamic):
    """eps = 0 makes sigma = h/h = 1, so n intervals of one CN step each are the
    plain path with n CN steps of T/n (up to the FFT round trips)."""
    f, mask, rmap = _case()
    N, T, beta, n = 16, 0.4, 2.0, 8
    out, _, _, _ = RO.restore(f, mask, N, T, beta, n, eps=0.0, dynamic=dynamic, rmap=rmap)
    want, _ = O.inpaint(f, mask, N, T, beta, n, rmap=rmap)
    assert _rel(out, want) < 1e-12


@pytest.mark.parametrize("dynamic", [False, True])
def test_one_interval_has_no_mix(dynamic):
    f, mask, rmap = _case(seed=5)
    N = 16
    out, _, join, _ = RO.restore(f, mask, N, 0.3, 1.5, 1, eps=0.7, dynamic=dynamic, substeps=4, rmap=rmap)
    want, _ = O.inpaint(f, mask, N, 0.3, 1.5, 4, rmap=rmap)
    assert _rel(out, want) < 1e-13
    assert set(np.unique(join)) <= {-1, 0}


def test_eps_changes_the_result():
    f, mask, rmap = _case(seed=6)
    a, *_ = RO.restore(f, mask, 16, 0.4, 2.0, 8, eps=0.5, rmap=rmap)
    b, _ = O.inpaint(f, mask, 16, 0.4, 2.0, 8, rmap=rmap)
    assert _rel(a, b) > 1e-3


@pytest.mark.parametrize("eps", [0.0, 0.3, 1.0])
def test_mix_sets_the_good_maximum_to_the_convex_combination(eps):
    rng = np.random.default_rng(1)
    N, M = 8, 12
    psi = rng.normal(0.2, 1.0, size=(N, M, M))
    psi[:, 0, :] = -np.abs(psi[:, 0, :])  # a row where h <= 0
    href = rng.uniform(0.0, 2.0, size=(M, M))
    good = rng.uniform(size=(M, M)) < 0.6
    mixed, h = RO.mix(psi, href, good, eps)
    assert np.array_equal(h, psi.max(axis=0))
    act = good & (h > 0)
    # the new maximum is eps href + (1 - eps) h
    np.testing.assert_allclose(mixed.max(axis=0)[act], (eps * href + (1 - eps) * h)[act], rtol=1e-14, atol=1e-15)
    # one factor for every orientation of a pixel
    ratio = mixed[:, act] / psi[:, act]
    np.testing.assert_allclose(ratio, np.broadcast_to(ratio[0], ratio.shape), rtol=1e-13)
    # bad pixels and good pixels without a positive maximum are untouched
    assert np.array_equal(mixed[:, ~act], psi[:, ~act])
    assert (~act & good).any() and (~good).any()


@pytest.mark.parametrize("dynamic", [False, True])
def test_degree_one_homogeneity(dynamic):
    """sigma and the DR comparison are scale free, the diffusion is linear and
    the orientation of c*f is that of f: restore(c f) = c restore(f)."""
    f, mask, rmap = _case(seed=7)
    a, _, ja, _ = RO.restore(f, mask, 16, 0.3, 2.0, 6, eps=0.5, dynamic=dynamic, rmap=rmap)
    b, _, jb, _ = RO.restore(2.5 * f, mask, 16, 0.3, 2.0, 6, eps=0.5, dynamic=dynamic, rmap=rmap)
    assert _rel(b, 2.5 * a) < 1e-13
    assert np.array_equal(ja, jb)


def _rot90(img):
    """f'[y][x] = f[(-x) mod M][y]: rotation of the periodic grid by +90 degrees."""
    M = img.shape[-1]
    idx = (-np.arange(M)) % M
    return np.swapaxes(img, -1, -2)[..., :, idx]


@pytest.mark.parametrize("dynamic", [False, True])
def test_rotation_equivariance(dynamic):
    """The operator commutes with the 90-degree rotation when orientations shift
    by N/4 (4 | N); the mix is per pixel and the DR neighbourhood is square, so
    both procedures commute with it too."""
    f, mask, rmap = _case(seed=8)
    N = 16
    a, _, ja, _ = RO.restore(f, mask, N, 0.3, 2.0, 6, eps=0.5, dynamic=dynamic, rmap=rmap)
    rrot = ((_rot90(rmap).astype(int) + N // 4) % N).astype(np.uint8)
    b, _, jb, _ = RO.restore(_rot90(f), _rot90(mask), N, 0.3, 2.0, 6, eps=0.5, dynamic=dynamic, rmap=rrot)
    assert _rel(b, _rot90(a)) < 1e-12
    assert np.array_equal(jb, _rot90(ja))


def test_dr_grows_and_differs_from_sr():
    f, mask, rmap = _case(seed=9)
    a, _, ja, info = RO.restore(f, mask, 16, 0.4, 2.0, 10, eps=0.5, dynamic=True, rmap=rmap)
    b, _, jb, _ = RO.restore(f, mask, 16, 0.4, 2.0, 10, eps=0.5, dynamic=False, rmap=rmap)
    assert (ja > 0).any(), "some bad pixels become good"
    assert np.array_equal(ja == 0, mask == 0) and np.array_equal(jb == 0, mask == 0)
    assert (jb == -1).sum() == mask.sum()
    assert _rel(a, b) > 1e-6
    assert info["min_margin"] > 0


def test_dr_with_imposed_updates_reproduces_itself():
    f, mask, rmap = _case(seed=10)
    a, _, ja, _ = RO.restore(f, mask, 16, 0.4, 2.0, 10, eps=0.5, dynamic=True, rmap=rmap)
    b, _, jb, info = RO.restore(f, mask, 16, 0.4, 2.0, 10, eps=0.5, dynamic=True, rmap=rmap, join_in=ja)
    assert np.array_equal(ja, jb) and info["flips"] == 0
    assert _rel(b, a) == 0.0


def _grid(bad_cells, hvals, M=6, hgood=9.0):
    good = np.ones((M, M), dtype=bool)
    h = np.full((M, M), hgood)
    for (y, x), v in zip(bad_cells, hvals):
        good[y, x] = False
        h[y, x] = v
    return good, h


def test_growth_rule_on_hand_worked_grids():
    """Worked by hand from the definition (3x3 neighbourhood, periodic,
    strict inequality, mean over the bad points only)."""
    # 2x2 bad block with h = 4, 1 / 1, 2: every bad neighbourhood holds all
    # four, mean 2; only 4 > 2 (2 > 2 fails: strict).
    good, h = _grid([(2, 2), (2, 3), (3, 2), (3, 3)], [4.0, 1.0, 1.0, 2.0])
    new, margin = RO.grow(good, h)
    assert sorted(zip(*np.nonzero(new))) == [(2, 2)]
    assert margin[3, 3] == 0.0 and margin[2, 2] == 2.0
    # 1x3 bad strip with h = 3, 1, 3: the ends see two bad points (mean 2) and
    # join, the middle sees all three (mean 7/3) and stays bad.
    good, h = _grid([(2, 1), (2, 2), (2, 3)], [3.0, 1.0, 3.0])
    new, _ = RO.grow(good, h)
    assert sorted(zip(*np.nonzero(new))) == [(2, 1), (2, 3)]
    # 3x3 bad block: its centre has no good neighbour, so it cannot join
    # however large its value; the ring's means include the centre's 100.
    cells = [(y, x) for y in (1, 2, 3) for x in (1, 2, 3)]
    good, h = _grid(cells, [100.0 if c == (2, 2) else 0.0 for c in cells])
    new, margin = RO.grow(good, h)
    assert not new.any()
    assert np.isnan(margin[2, 2])
    # neighbourhoods wrap around: (0, 0) and (0, 5) are neighbours
    good, h = _grid([(0, 0), (0, 5)], [2.0, 1.0])
    new, _ = RO.grow(good, h)
    assert sorted(zip(*np.nonzero(new))) == [(0, 0)]


def test_growth_rule_counts_edge_and_corner_neighbours():
    """One good pixel at (2, 2) in a bad 6x6 grid: its 8 neighbours are the
    boundary.  (1, 2) touches it through an edge only, (1, 1) through a corner
    only; with h = 5 there and 0 on every other bad pixel, each sees 7 other
    bad points plus itself (mean 5/8) and joins; (3, 3), with h = 0 = its
    mean, does not."""
    M = 6
    good = np.zeros((M, M), dtype=bool)
    good[2, 2] = True
    h = np.zeros((M, M))
    h[1, 2] = 5.0
    h[1, 1] = 5.0
    new, margin = RO.grow(good, h)
    # (1, 2)'s neighbourhood holds (1, 1) as well: mean (5 + 5)/8
    assert sorted(zip(*np.nonzero(new))) == [(1, 1), (1, 2)]
    assert margin[1, 2] == 5.0 - 10.0 / 8.0
    assert margin[3, 3] == 0.0 and not new[3, 3]
    assert np.isnan(margin[0, 0])  # not on the boundary


def test_dr_with_two_intervals_equals_sr():
    """With two intervals the only mix is at t_1, where the points that join G
    are mixed towards their own current value (sigma = 1), exactly as SR
    leaves bad points alone: DR and SR agree."""
    f, mask, rmap = _case(seed=12)
    a, _, ja, _ = RO.restore(f, mask, 16, 0.2, 2.0, 2, eps=0.6, dynamic=True, rmap=rmap)
    b, *_ = RO.restore(f, mask, 16, 0.2, 2.0, 2, eps=0.6, dynamic=False, rmap=rmap)
    assert (ja == 1).any()
    assert _rel(a, b) < 1e-14


def test_growth_rule_properties():
    rng = np.random.default_rng(4)
    for _ in range(20):
        M = 9
        good = rng.uniform(size=(M, M)) < 0.5
        h = rng.normal(size=(M, M))
        new, margin = RO.grow(good, h)
        assert not (new & good).any()
        # every new point has a good 8-neighbour and beats its bad mean
        for y, x in zip(*np.nonzero(new)):
            nb = [((y + dy) % M, (x + dx) % M) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
            assert any(good[p] for p in nb if p != (y, x))
            bad_vals = [h[p] for p in nb if not good[p]]
            assert h[y, x] > np.mean(bad_vals)
        assert np.all(np.isfinite(margin) == (~good & ~np.isnan(margin)))


def _table1_rows():
    rows = []
    with open(os.path.join(GOLDEN, "table1_parameters.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            name, alpha, T, n, eps, w, pct = line.split()
            rows.append((name, float(alpha), float(T), int(n), float(eps), int(w), int(pct)))
    return rows


def test_table1_workloads_follow_the_printed_parameters():
    """synth.table1_case reproduces each printed row: alpha -> beta_N at N = 30
    by relation (relation), T = T_p / 2 (the clock reading), n, eps, the line
    width, and the corruption within 2 points of the printed percentage."""
    rows = _table1_rows()
    assert [r[0] for r in rows] == list(synth.TABLE1)
    for name, alpha, Tp, n, eps, w, pct in rows:
        c = synth.table1_case(name)
        assert c["M"] == 256 and c["N"] == 30
        assert abs(c["beta"] * (2 * np.pi / 30) ** 2 - alpha) < 1e-13
        assert c["T"] == Tp / 2 and c["n"] == n and c["eps"] == eps and c["width"] == w
        assert abs(100 * c["corruption"] - pct) < 2.0
        assert c["f"][c["mask"] == 0].min() > 0.0  # the procedures assume f > 0 on G
        assert c["dynamic"] == (not name.startswith("fig2"))
