"""Pins of the oracle's polar quadtree (Sec. 2-D, Sec. 4-A): two independent
constructions agree, brute force on small inputs, structural invariants,
cell diameters by dense sampling, and the shrink factor remark of Sec. 4-A."""
import numpy as np
import pytest

import oracle
from paper_2401_13708_amd import synth

L = 20


def _polar32(Y):
    Ys = Y.astype(np.float32).astype(np.float64)
    r = np.sqrt(Ys[:, 0] ** 2 + Ys[:, 1] ** 2)
    p = np.arctan2(Ys[:, 1], Ys[:, 0])
    p = np.where(p < 0, p + 2 * np.pi, p)
    return r, p


def _inputs():
    out = []
    for st in ["init", "early", "mid", "late", "edge"]:
        out.append((st, synth.disk_state(257, st, seed=3).astype(np.float64)))
    Y = synth.disk_state(200, "mid", seed=4).astype(np.float64)
    Y[50:60] = Y[5]          # a block of duplicates
    Y[100] = Y[101]
    out.append(("dups", Y))
    out.append(("two", np.array([[0.1, 0.2], [-0.3, 0.05]])))
    out.append(("same_radius", np.stack([0.5 * np.cos(np.arange(64) * 0.1),
                                         0.5 * np.sin(np.arange(64) * 0.1)], 1)))
    return out


@pytest.mark.parametrize("name,Y", _inputs())
def test_insertion_equals_partition(name, Y):
    a = oracle.Tree(Y, L, "insert").export()
    b = oracle.Tree(Y, L, "partition").export()
    for key in ("count", "depth", "first", "next", "perm"):
        assert np.array_equal(a[key], b[key]), key
    assert np.array_equal(a["mid"], b["mid"])
    assert np.array_equal(a["r_cell"], b["r_cell"])


def _brute_nodes(Y, max_depth):
    """Node set from digit strings: a cell at depth l is a node iff it is
    non-empty and its parent holds at least two points (or it is the root)."""
    r, p = _polar32(Y)
    n = Y.shape[0]
    keys = []
    for i in range(n):
        lo, hi, plo, phi = r.min(), r.max(), 0.0, 2 * np.pi
        dig = []
        for _ in range(max_depth):
            mr, mp = (lo + hi) * 0.5, (plo + phi) * 0.5
            rb, pb = int(r[i] >= mr), int(p[i] >= mp)
            dig.append(2 * rb + pb)
            lo, hi = (mr, hi) if rb else (lo, mr)
            plo, phi = (mp, phi) if pb else (plo, mp)
        keys.append(tuple(dig))
    nodes = {(): n}
    for lvl in range(1, max_depth + 1):
        for i in range(n):
            pre = keys[i][:lvl]
            parent = keys[i][:lvl - 1]
            cnt_parent = sum(1 for k in keys if k[:lvl - 1] == parent)
            if cnt_parent >= 2:
                nodes[pre] = sum(1 for k in keys if k[:lvl] == pre)
    order = sorted(nodes.keys())    # lexicographic = pre-order, children by digit
    return [(len(k), nodes[k]) for k in order]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_small_tree_matches_brute_force(seed):
    Y = synth.disk_state(48, ["early", "mid", "late"][seed], n_clusters=3, seed=seed).astype(np.float64)
    Y[7] = Y[8]
    e = oracle.Tree(Y, 8).export()
    got = list(zip(e["depth"].tolist(), e["count"].tolist()))
    assert got == _brute_nodes(Y, 8)


@pytest.mark.parametrize("name,Y", _inputs())
def test_structural_invariants(name, Y):
    e = oracle.Tree(Y, L).export()
    n, m = Y.shape[0], e["count"].size
    assert sorted(e["perm"].tolist()) == list(range(n))
    assert e["count"][0] == n and e["depth"][0] == 0 and e["next"][0] == m
    for k in range(m):
        leaf = e["next"][k] == k + 1
        if leaf:
            assert e["count"][k] == 1 or e["depth"][k] == L
            if e["count"][k] > 1:   # only identical positions share a deepest leaf
                pts = Y[e["perm"][e["first"][k]:e["first"][k] + e["count"][k]]].astype(np.float32)
                r, p = _polar32(pts.astype(np.float64))
        else:
            assert e["count"][k] >= 2
            c, tot = k + 1, 0
            while c < e["next"][k]:
                assert e["depth"][c] == e["depth"][k] + 1
                assert e["first"][c] == e["first"][k] + tot
                tot += e["count"][c]
                b, bc = e["bounds"][k], e["bounds"][c]
                assert b[0] <= bc[0] <= bc[1] <= b[1] and b[2] <= bc[2] <= bc[3] <= b[3]
                assert e["r_cell"][c] <= e["r_cell"][k] * (1 + 1e-12)
                c = e["next"][c]
            assert tot == e["count"][k]
    # points lie in their leaf cells
    r, p = _polar32(Y)
    for k in range(m):
        pts = e["perm"][e["first"][k]:e["first"][k] + e["count"][k]]
        b = e["bounds"][k]
        assert np.all((r[pts] >= b[0]) & (r[pts] <= b[1]) & (p[pts] >= b[2]) & (p[pts] <= b[3]))


def test_cell_diameter_by_sampling():
    # the stored diameter bounds every pairwise distance inside the cell and is
    # attained (up to sampling) by points of the cell
    Y = synth.disk_state(400, "late", seed=5).astype(np.float64)
    e = oracle.Tree(Y, L).export()
    g = np.random.default_rng(0)
    ks = [k for k in range(e["count"].size) if e["next"][k] != k + 1]
    for k in ks[:: max(1, len(ks) // 40)]:
        rlo, rhi, plo, phi = e["bounds"][k]
        rr = np.concatenate([[rlo, rhi], g.uniform(rlo, rhi, 60)])
        pp = np.concatenate([[plo, phi], g.uniform(plo, phi, 60)])
        R, P = np.meshgrid(rr, pp)
        pts = np.stack([(R * np.cos(P)).ravel(), (R * np.sin(P)).ravel()], 1)
        sub = pts[g.choice(len(pts), 300, replace=False)]
        sub = np.concatenate([sub, pts[:2], pts[-2:], [[rlo * np.cos(plo), rlo * np.sin(plo)],
                                                        [rhi * np.cos(phi), rhi * np.sin(phi)],
                                                        [rhi * np.cos(plo), rhi * np.sin(plo)]]])
        a, b = sub[:, None, :], sub[None, :, :]
        num = 2 * np.sum((a - b) ** 2, -1)
        den = (1 - np.sum(a * a, -1)) * (1 - np.sum(b * b, -1))
        dmax = np.arccosh(1 + num / den).max()
        assert dmax <= e["r_cell"][k] * (1 + 1e-9)
        assert dmax >= 0.9 * e["r_cell"][k]


def test_shrink_factor_approaches_half():
    # Sec. 4-A: the longest distance in a cell shrinks by a factor that
    # approaches 0.5 after a few levels (a preliminary observation; soft pin)
    Y = synth.disk_state(4000, "mid", seed=6).astype(np.float64)
    e = oracle.Tree(Y, L).export()
    ratios = {}
    for k in range(e["count"].size):
        if e["next"][k] == k + 1:
            continue
        c = k + 1
        while c < e["next"][k]:
            ratios.setdefault(int(e["depth"][c]), []).append(e["r_cell"][c] / e["r_cell"][k])
            c = e["next"][c]
    deep = [np.median(v) for d, v in ratios.items() if 5 <= d <= 12 and len(v) > 20]
    assert deep and all(0.4 < x < 0.6 for x in deep), deep


def test_root_diameter_closed_form():
    # the root is an annulus; its diameter is the antipodal pair on the outer circle
    Y = synth.disk_state(100, "mid", seed=8).astype(np.float64)
    e = oracle.Tree(Y, L).export()
    rhi = e["bounds"][0][1]
    assert e["r_cell"][0] == pytest.approx(4 * np.arctanh(rhi), rel=1e-12)


def test_midpoints_are_einstein_midpoints_of_cells():
    Y = synth.disk_state(300, "late", seed=9).astype(np.float64)
    e = oracle.Tree(Y, L).export()
    for k in range(0, e["count"].size, 7):
        pts = Y[e["perm"][e["first"][k]:e["first"][k] + e["count"][k]]]
        # independent evaluation of eq. (11): Klein coordinates, gamma weights
        v = 2 * pts / (1 + np.sum(pts * pts, 1, keepdims=True))
        gm = 1 / np.sqrt(1 - np.sum(v * v, 1))
        K = (gm[:, None] * v).sum(0) / gm.sum()
        m = K / (1 + np.sqrt(1 - K @ K))
        # the printed form divides by sqrt(1 - |v|^2), which cancels near the rim
        tol = 1e-12 + 1e-16 / np.min(1 - np.sum(pts * pts, 1)) ** 2
        assert np.allclose(e["mid"][k], m, rtol=tol, atol=1e-15)


# ---------------------------------------------------------------- eq. (9)
def test_equal_area_mid_is_the_printed_formula():
    # eq. (9) in the hyperbolic radius rho = 2 artanh(r), evaluated literally
    g = np.random.default_rng(7)
    for lo, hi in [(0.0, 0.5), (0.1, 0.2), (1e-4, 2e-4), (0.9, 0.99999), (0.3, 0.3000001)]:
        rlo, rhi = 2 * np.arctanh(lo), 2 * np.arctanh(hi)
        mid_rho = np.arccosh((np.cosh(rhi) + np.cosh(rlo)) / 2)
        want = np.tanh(mid_rho / 2)
        assert oracle.radial_mid(lo, hi, 1) == pytest.approx(want, rel=1e-9), (lo, hi)
    for _ in range(200):
        lo, hi = np.sort(g.uniform(0, 0.999, 2))
        rlo, rhi = 2 * np.arctanh(lo), 2 * np.arctanh(hi)
        want = np.tanh(np.arccosh((np.cosh(rhi) + np.cosh(rlo)) / 2) / 2)
        assert oracle.radial_mid(lo, hi, 1) == pytest.approx(want, rel=1e-9)
    assert oracle.radial_mid(0.2, 0.6, 0) == 0.4


def test_equal_area_mid_halves_the_hyperbolic_area():
    # the area inside hyperbolic radius rho is 2 pi (cosh rho - 1), and
    # cosh rho = (1 + r^2) / (1 - r^2): both halves of the annulus are equal
    ch = lambda r: (1 + r * r) / (1 - r * r)
    g = np.random.default_rng(8)
    for _ in range(200):
        lo, hi = np.sort(g.uniform(0, 0.99, 2))
        m = oracle.radial_mid(lo, hi, 1)
        assert lo <= m <= hi
        inner, outer = ch(m) - ch(lo), ch(hi) - ch(m)
        assert inner == pytest.approx(outer, rel=1e-9, abs=1e-15)
    # the split lies outside the equal-length mid (area grows with the radius)
    assert oracle.radial_mid(0.0, 0.9, 1) > 0.45


@pytest.mark.parametrize("name,Y", _inputs())
def test_equal_area_insertion_equals_partition(name, Y):
    a = oracle.Tree(Y, L, "insert", split_rule=1).export()
    b = oracle.Tree(Y, L, "partition", split_rule=1).export()
    for key in ("count", "depth", "first", "next", "perm"):
        assert np.array_equal(a[key], b[key]), key
    # cells split at the equal-area radius
    for k in range(a["count"].size):
        if a["next"][k] != k + 1 and a["depth"][k] < L:
            rlo, rhi = a["bounds"][k][:2]
            c = k + 1
            while c < a["next"][k]:
                blo, bhi = a["bounds"][c][:2]
                m = oracle.radial_mid(rlo, rhi, 1)
                assert (blo, bhi) in ((rlo, m), (m, rhi))
                c = a["next"][c]


def test_equal_area_small_tree_matches_brute_force():
    Y = synth.disk_state(48, "late", n_clusters=3, seed=9).astype(np.float64)
    r, p = _polar32(Y)
    ch = lambda x: (1 + x * x) / (1 - x * x)
    n, depth = Y.shape[0], 8
    keys = []
    for i in range(n):
        lo, hi, plo, phi = r.min(), r.max(), 0.0, 2 * np.pi
        dig = []
        for _ in range(depth):
            # equal-area split found by bisection on the area balance
            a, b = lo, hi
            for _ in range(200):
                m = 0.5 * (a + b)
                if ch(m) - ch(lo) < ch(hi) - ch(m):
                    a = m
                else:
                    b = m
            mr = oracle.radial_mid(lo, hi, 1)
            assert abs(mr - 0.5 * (a + b)) <= 1e-12 * max(1.0, hi)
            mp = (plo + phi) * 0.5
            rb, pb = int(r[i] >= mr), int(p[i] >= mp)
            dig.append(2 * rb + pb)
            lo, hi = (mr, hi) if rb else (lo, mr)
            plo, phi = (mp, phi) if pb else (plo, mp)
        keys.append(tuple(dig))
    nodes = {(): n}
    for lvl in range(1, depth + 1):
        for i in range(n):
            parent = keys[i][:lvl - 1]
            if sum(1 for k in keys if k[:lvl - 1] == parent) >= 2:
                nodes[keys[i][:lvl]] = sum(1 for k in keys if k[:lvl] == keys[i][:lvl])
    want = [(len(k), nodes[k]) for k in sorted(nodes)]
    e = oracle.Tree(Y, depth, split_rule=1).export()
    assert list(zip(e["depth"].tolist(), e["count"].tolist())) == want


# ---------------------------------------------------------------- angular split
def test_sign_of_the_split_test_is_exact():
    # the angular decision is the sign of c y - s x with single-precision c,
    # s, x, y evaluated in double: both products are exact (48 significant
    # bits) and one rounding cannot change the sign of the difference.
    # Checked against rational arithmetic on points within a few units in
    # the last place of the ray (c, s).
    from fractions import Fraction
    g = synth.rng(71)
    bad = 0
    for _ in range(4000):
        a = g.uniform(0.0, 2.0 * np.pi)
        c, s = np.float32(np.cos(a)), np.float32(np.sin(a))
        r = g.uniform(1e-4, 0.999)
        x, y = np.float32(r * np.cos(a)), np.float32(r * np.sin(a))
        for _ in range(int(g.integers(0, 4))):
            x = np.nextafter(x, np.float32(g.choice([-1.0, 1.0])))
        fast = float(c) * float(y) - float(s) * float(x)
        exact = Fraction(float(c)) * Fraction(float(y)) - Fraction(float(s)) * Fraction(float(x))
        bad += (fast >= 0.0) != (exact >= 0)
        bad += (fast == 0.0) != (exact == 0)
    assert bad == 0


def _leaf_bounds_of_points(e):
    # bounds of the leaf holding each point (a leaf is a node with next = k + 1)
    m = e["count"].size
    out = {}
    for k in range(m):
        if e["next"][k] == k + 1:
            for a in range(e["first"][k], e["first"][k] + e["count"][k]):
                out[int(e["perm"][a])] = e["bounds"][k]
    return out


def test_points_on_split_rays_go_to_the_upper_half():
    # points exactly on the rays at multiples of pi/4 (coordinates exactly
    # representable, x = +-y on the diagonals): the tree sends a point on a
    # cell's split ray to the upper half, as phi >= (min + max) / 2 does, so
    # the leaf holding a point at angle phi has p_lo <= phi < p_hi
    rad = np.array([0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8], dtype=np.float64)
    dirs = [(1, 0), (1, 1), (0, 1), (-1, 1), (-1, 0), (-1, -1), (0, -1), (1, -1)]
    Y = np.array([(r * dx, r * dy) for dx, dy in dirs for r in rad])
    phis = np.array([k * np.pi / 4 for k in range(8) for _ in rad])
    for depth in (6, 20):
        e = oracle.Tree(Y, depth).export()
        lb = _leaf_bounds_of_points(e)
        for i in range(Y.shape[0]):
            plo, phi = lb[i][2], lb[i][3]
            assert plo <= phis[i] + 1e-15 and phis[i] < phi - 1e-15, (i, phis[i], plo, phi)


def test_near_ray_points_insertion_equals_partition_and_brute_force_away_from_rays():
    Y = synth.near_split_rays().astype(np.float64)
    a = oracle.Tree(Y, L, "insert").export()
    b = oracle.Tree(Y, L, "partition").export()
    for key in ("count", "depth", "first", "next", "perm"):
        assert np.array_equal(a[key], b[key]), key
    # every point lies in its leaf's angular range up to the rounding of the
    # split rays (a few 1e-8 rad)
    r, p = _polar32(Y)
    lb = _leaf_bounds_of_points(a)
    for i in range(Y.shape[0]):
        plo, phi = lb[i][2], lb[i][3]
        assert plo - 1e-7 <= p[i] <= phi + 1e-7
