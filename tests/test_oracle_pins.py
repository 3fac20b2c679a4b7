"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed
forms, hand-derived fixtures, exact rational brute force, autograd of an
independent formulation, finite differences, or special cases that reduce to
a textbook result.  None of them needs a GPU.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# ----------------------------------------------------------------------------
# ray / box clip
# ----------------------------------------------------------------------------
BMIN = np.array([-1.5, -1.5, -1.5], np.float32)
BMAX = np.array([1.5, 1.5, 1.5], np.float32)


def test_clip_axis_aligned_exact():
    o = np.array([[-3, 0.25, 0.5], [3, 0.25, 0.5], [0.5, -4, 0.0], [-3, 2.0, 0.0]], np.float32)
    d = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [1, 0, 0]], np.float32)
    tn, tf = oracle.clip(o, d, BMIN, BMAX)
    assert tn[0] == 1.5 and tf[0] == 4.5
    assert tn[1] == 1.5 and tf[1] == 4.5
    assert tn[2] == 2.5 and tf[2] == 5.5
    assert not tn[3] < tf[3]  # passes above the box: miss


def test_clip_inside_and_near_plane():
    g = scenes.rng(11)
    o = g.uniform(-1, 1, (64, 3)).astype(np.float32)
    d = g.standard_normal((64, 3))
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    tn, tf = oracle.clip(o, d, BMIN, BMAX, near=0.0)
    assert np.all(tn == 0.0)
    exit_pt = o.astype(np.float64) + tf[:, None].astype(np.float64) * d
    np.testing.assert_allclose(np.abs(exit_pt).max(axis=1), 1.5, rtol=1e-6)
    tn2, _ = oracle.clip(o, d, BMIN, BMAX, near=0.25)
    assert np.all(tn2 == np.float32(0.25))


def test_clip_chord_through_centre():
    # rays aimed at the box centre: chord = 2 h / max_a |d_a|
    g = scenes.rng(12)
    d = g.standard_normal((256, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = -4.0 * d
    tn, tf = oracle.clip(o.astype(np.float32), d.astype(np.float32), BMIN, BMAX)
    chord = 2 * 1.5 / np.abs(d).max(axis=1)
    np.testing.assert_allclose(tf.astype(np.float64) - tn, chord, rtol=2e-6, atol=2e-6)
    entry = o + tn[:, None].astype(np.float64) * d
    np.testing.assert_allclose(np.abs(entry).max(axis=1), 1.5, rtol=2e-6)


def test_clip_ray_in_face_plane_parallel_misses():
    # a ray lying exactly in a face plane and parallel to it is a miss (reading)
    o = np.array([[-3, 1.5, 0.0], [-3, -1.5, 0.0]], np.float32)
    d = np.array([[1, 0, 0], [1, 0, 0]], np.float32)
    tn, tf = oracle.clip(o, d, BMIN, BMAX)
    assert not np.any(tn < tf)


# ----------------------------------------------------------------------------
# march (dense definition)
# ----------------------------------------------------------------------------
def test_march_golden_axis_ray():
    g = load_golden("axis_ray_march.json")
    res = g["res"]
    occ = np.zeros(res ** 3, bool)
    occ[g["occupied_cells"]] = True
    bits = scenes.pack_bits(occ)
    o = np.array([g["ray_o"]], np.float32)
    d = np.array([g["ray_d"]], np.float32)
    out = oracle.march(o, d, bits, res, half_extent0=g["half_extent"], dt0=g["dt"])
    assert out["t0"].tolist() == g["expected_t0"]
    assert out["t1"].tolist() == g["expected_t1"]
    full = oracle.march(o, d, scenes.pack_bits(np.ones(res ** 3, bool)), res,
                        half_extent0=g["half_extent"], dt0=g["dt"])
    assert full["total"] == g["full_grid_count"]
    assert full["t0"][0] == g["t_near"] and full["t1"][-1] == g["t_far"]


def test_march_golden_cascade():
    g = load_golden("cascade_ray_march.json")
    res, L = g["res"], g["n_levels"]
    bits = np.concatenate([scenes.pack_bits(np.ones(res ** 3, bool))] * L)
    out = oracle.march(np.array([g["ray_o"]], np.float32), np.array([g["ray_d"]], np.float32),
                       bits, res, n_levels=L, half_extent0=g["half_extent0"], dt0=g["dt0"],
                       want_level=True)
    assert out["t0"].tolist() == g["expected_t0"]
    assert out["t1"].tolist() == g["expected_t1"]
    assert out["level"].tolist() == g["expected_level"]


def test_march_empty_grid_gives_nothing():
    o, d = scenes.sphere_rays(512, seed=21)
    out = oracle.march(o, d, np.zeros(64 ** 3 // 32, np.uint32), 64, dt0=0.01)
    assert out["total"] == 0


def test_march_full_grid_count_closed_form():
    # every lattice midpoint inside the chord is kept: count = ceil((tf-tn)/dt - 1/2)
    o, d = scenes.sphere_rays(2000, seed=22)
    dt = 0.0123
    out = oracle.march(o, d, scenes.pack_bits(np.ones(16 ** 3, bool)), 16, dt0=dt)
    tn, tf = oracle.clip(o, d, BMIN, BMAX)
    hit = tn < tf
    q = (tf.astype(np.float64) - tn) / np.float64(np.float32(dt)) - 0.5
    expect = np.where(hit, np.ceil(q), 0)
    near_int = np.abs(q - np.round(q)) < 1e-4  # binary32 midpoint may land either side
    ok = (out["counts"] == expect) | near_int
    assert ok.all()
    assert (~near_int[hit]).sum() > 1900 * hit.mean()


def _exact_cells(o, d, tn, tf, dt, res, h):
    """Exact-rational lattice walk: (k, cell or None if ambiguous) for each midpoint."""
    O = [Fraction(float(v)) for v in o]
    D = [Fraction(float(v)) for v in d]
    a, b, step = Fraction(float(tn)), Fraction(float(tf)), Fraction(float(dt))
    lo = Fraction(float(-h))
    size = Fraction(2 * h) / res
    out = []
    k = 0
    while True:
        m = a + (k + Fraction(1, 2)) * step
        if m >= b:
            # a midpoint within a hair of t_far is binary32-ambiguous
            if m - b < Fraction(1, 10 ** 6) * step:
                out.append((k, None))
            break
        cell = []
        amb = False
        for c in range(3):
            u = (O[c] + m * D[c] - lo) / size
            fl = math.floor(u)
            if abs(u - fl) < Fraction(1, 10 ** 4) or abs(u - fl - 1) < Fraction(1, 10 ** 4):
                amb = True
            cell.append(min(max(fl, 0), res - 1))
        if b - m < Fraction(1, 10 ** 6) * step:
            amb = True
        out.append((k, None if amb else cell[0] + res * (cell[1] + res * cell[2])))
        k += 1
    return out


@pytest.mark.parametrize("res", [2, 3, 4, 8])
def test_march_matches_exact_rational_brute_force(res):
    g = scenes.rng(100 + res)
    occ = g.random(res ** 3) < 0.45
    bits = scenes.pack_bits(np.concatenate([occ, np.zeros((-res ** 3) % 32, bool)]))
    n = 40
    o, d = scenes.sphere_rays(n, radius=2.5, target_half=1.2, seed=200 + res)
    dt = np.float32(0.037)
    out = oracle.march(o, d, bits, res, dt0=float(dt))
    tn, tf = oracle.clip(o, d, BMIN, BMAX)
    checked = 0
    for r in range(n):
        s, c = out["packed_info"][r]
        got_t0 = out["t0"][s:s + c]
        if not tn[r] < tf[r]:
            assert c == 0
            continue
        exact = _exact_cells(o[r], d[r], tn[r], tf[r], dt, res, 1.5)
        # recover the lattice index of each emitted sample from its t0
        got_k = np.rint((got_t0.astype(np.float64) - tn[r]) / np.float64(dt)).astype(int)
        got = set(got_k.tolist())
        for k, cell in exact:
            if cell is None:
                continue
            checked += 1
            assert (k in got) == bool(occ[cell]), (r, k, cell)
        # emitted intervals: [tn + k dt, min(tn + (k+1) dt, tf)] up to binary32 rounding
        np.testing.assert_allclose(got_t0, tn[r] + got_k * np.float64(dt), rtol=1e-6, atol=1e-6)
        np.testing.assert_allclose(out["t1"][s:s + c],
                                   np.minimum(tn[r] + (got_k + 1) * np.float64(dt), tf[r]),
                                   rtol=1e-6, atol=1e-6)
    assert checked > 100


def test_march_grid_layout_x_fastest():
    # a single occupied cell at (x,y,z) = (3,1,0) of a 4^3 grid; ray along +x at its row
    res = 4
    occ = np.zeros(res ** 3, bool)
    occ[3 + res * (1 + res * 0)] = True
    o = np.array([[-3.0, -1.5 + 0.75 * 1.5, -1.5 + 0.75 * 0.5]], np.float32)
    d = np.array([[1.0, 0.0, 0.0]], np.float32)
    out = oracle.march(o, d, scenes.pack_bits(occ), res, dt0=0.25)
    # x-cell 3 covers x in [0.75, 1.5): t in [3.75, 4.5): k = 9, 10, 11
    assert out["t0"].tolist() == [3.75, 4.0, 4.25]


def test_march_cap_and_prefix():
    o, d = scenes.sphere_rays(300, seed=31)
    bits = scenes.occupancy_bits(scenes.blob_field(8), 32)
    full = oracle.march(o, d, bits, 32, dt0=0.01)
    cap = oracle.march(o, d, bits, 32, dt0=0.01, max_per_ray=7)
    assert np.array_equal(cap["counts"], np.minimum(full["counts"], 7))
    for r in range(300):
        s0, c0 = full["packed_info"][r]
        s1, c1 = cap["packed_info"][r]
        assert np.array_equal(cap["t0"][s1:s1 + c1], full["t0"][s0:s0 + c1])


def test_cascade_with_empty_outer_levels_equals_inner_march():
    fld = scenes.blob_field(8)
    res = 16
    lvl0 = scenes.occupancy_bits(fld, res)
    empty = np.zeros_like(lvl0)
    o, d = scenes.sphere_rays(500, radius=5.0, seed=41)
    casc = oracle.march(o, d, np.concatenate([lvl0, empty, empty]), res, n_levels=3, dt0=0.01)
    plain = oracle.march(o, d, lvl0, res, n_levels=1, dt0=0.01)
    # the level-0 segment of the cascade starts at the inner cube's entry: same lattice
    assert np.array_equal(casc["counts"], plain["counts"])
    assert np.array_equal(casc["t0"], plain["t0"]) and np.array_equal(casc["t1"], plain["t1"])


def test_cascade_full_levels_cover_chord():
    # all levels full: the intervals tile [t_near, t_far] of the outer cube except for
    # slivers shorter than half a step at segment ends
    res = 8
    full = scenes.pack_bits(np.ones(res ** 3, bool))
    o, d = scenes.sphere_rays(200, radius=20.0, target_half=2.0, seed=42)
    out = oracle.march(o, d, np.concatenate([full] * 3), res, n_levels=3, dt0=0.05,
                       want_level=True)
    bmin = np.full(3, -6.0, np.float32)
    tn, tf = oracle.clip(o, d, bmin, -bmin)
    for r in range(200):
        s, c = out["packed_info"][r]
        if not tn[r] < tf[r]:
            assert c == 0
            continue
        t0 = out["t0"][s:s + c].astype(np.float64)
        t1 = out["t1"][s:s + c].astype(np.float64)
        lv = out["level"][s:s + c]
        assert t0[0] == tn[r]
        assert np.all(t1 > t0) and np.all(t0[1:] >= t1[:-1] - 1e-6)
        gaps = t0[1:] - t1[:-1]
        step = 0.05 * 2.0 ** lv[:-1]
        assert np.all(gaps < 0.5 * step + 1e-5)
        assert abs(t1[-1] - tf[r]) < 0.5 * 0.05 * 4 + 1e-5
        # step doubles per level, level never skips one between neighbours
        assert np.all(np.abs(np.diff(lv)) <= 1)


# ----------------------------------------------------------------------------
# render forward
# ----------------------------------------------------------------------------
def _uniform_ray(n, L, sigma, colour):
    dt = L / n
    t0 = (np.arange(n) * dt).astype(np.float32)
    t1 = (np.arange(1, n + 1) * dt).astype(np.float32)
    return (np.array([[0, n]], np.int32), t0, t1, np.full(n, sigma, np.float32),
            np.tile(np.asarray(colour, np.float32), (n, 1)))


def test_render_constant_density_closed_forms():
    # Eq. 2: constant sigma gives T(t) = exp(-sigma t) and opacity 1 - exp(-sigma L)
    n, L, sig = 100, 2.0, 1.7
    info, t0, t1, s, c = _uniform_ray(n, L, sig, [0.2, 0.5, 0.9])
    out = oracle.render_fwd(info, t0, t1, s, c, want_weights=True)
    sig64 = float(np.float32(sig))
    dt = t1.astype(np.float64) - t0
    Lr = float(t1[-1])
    assert out["opacity"][0] == pytest.approx(1 - math.exp(-sig64 * Lr), rel=1e-12)
    np.testing.assert_allclose(out["rgb"][0], np.float32([0.2, 0.5, 0.9]) * out["opacity"][0],
                               rtol=1e-12)
    T = np.exp(-sig64 * t0.astype(np.float64))
    np.testing.assert_allclose(out["weights"], T * (1 - np.exp(-sig64 * dt)), rtol=1e-10)
    # depth: sum_i q^i (1-q) m_i with q = exp(-sigma dt), m_i = (i+1/2) dt (uniform dt)
    q = math.exp(-sig64 * (L / n))
    i = np.arange(n)
    closed = (1 - q) * (L / n) * (np.sum(i * q ** i) + 0.5 * np.sum(q ** i))
    geo = q * (1 - n * q ** (n - 1) + (n - 1) * q ** n) / (1 - q) ** 2
    assert np.sum(i * q ** i) == pytest.approx(geo, rel=1e-12)
    assert out["depth"][0] == pytest.approx(closed, rel=1e-6)


def test_render_weights_sum_to_one_minus_final_transmittance():
    g = scenes.rng(51)
    counts = g.integers(0, 60, size=200).astype(np.int32)
    info, S = oracle.exclusive_scan(counts)
    t0 = np.concatenate([np.sort(g.uniform(0, 3, c)).astype(np.float32) for c in counts])
    t1 = (t0 + g.uniform(0.001, 0.05, S)).astype(np.float32)
    sig = g.exponential(5.0, S).astype(np.float32)
    rgb = g.random((S, 3)).astype(np.float32)
    out = oracle.render_fwd(info, t0, t1, sig, rgb, want_weights=True)
    tau = sig.astype(np.float64) * (t1.astype(np.float64) - t0)
    for r in range(200):
        s, c = info[r]
        Tfin = math.exp(-tau[s:s + c].sum())
        assert out["weights"][s:s + c].sum() == pytest.approx(1 - Tfin, rel=1e-12, abs=1e-15)
        assert out["opacity"][r] == pytest.approx(1 - Tfin, rel=1e-12, abs=1e-15)


def test_render_single_sample_empty_ray_and_background():
    info = np.array([[0, 1], [1, 0]], np.int32)
    t0 = np.array([1.0], np.float32)
    t1 = np.array([1.25], np.float32)
    s = np.array([3.0], np.float32)
    c = np.array([[1.0, 0.5, 0.25]], np.float32)
    bg = np.array([[0.1, 0.2, 0.3], [0.7, 0.8, 0.9]], np.float32)
    out = oracle.render_fwd(info, t0, t1, s, c, bg=bg)
    a = 1 - math.exp(-0.75)
    assert out["opacity"][0] == pytest.approx(a, rel=1e-14)
    assert out["depth"][0] == pytest.approx(a * 1.125, rel=1e-14)
    np.testing.assert_allclose(out["rgb"][0], a * c[0] + (1 - a) * bg[0].astype(np.float64),
                               rtol=1e-7)
    assert out["opacity"][1] == 0 and out["depth"][1] == 0
    np.testing.assert_allclose(out["rgb"][1], bg[1], rtol=0)


# ----------------------------------------------------------------------------
# render backward
# ----------------------------------------------------------------------------
def _random_packed(seed, n_rays=40, max_count=30):
    g = scenes.rng(seed)
    counts = g.integers(0, max_count, size=n_rays).astype(np.int32)
    info, S = oracle.exclusive_scan(counts)
    t0 = np.concatenate([np.sort(g.uniform(0, 2, c)) for c in counts]).astype(np.float32)
    t1 = (t0 + g.uniform(0.01, 0.1, S)).astype(np.float32)
    sig = g.exponential(3.0, S).astype(np.float32)
    rgb = g.random((S, 3)).astype(np.float32)
    return info, t0, t1, sig, rgb, g


def _torch_render(info, t0, t1, sig, rgb, bg=None):
    """Independent formulation: torch cumsum + exp, differentiated by autograd."""
    import torch
    outs = []
    for r in range(info.shape[0]):
        s, c = int(info[r, 0]), int(info[r, 1])
        delta = torch.as_tensor(t1[s:s + c], dtype=torch.float64) - torch.as_tensor(
            t0[s:s + c], dtype=torch.float64)
        tau = sig[s:s + c] * delta
        T = torch.exp(-(torch.cumsum(tau, 0) - tau))
        w = T * (1 - torch.exp(-tau))
        mid = 0.5 * (torch.as_tensor(t0[s:s + c], dtype=torch.float64)
                     + torch.as_tensor(t1[s:s + c], dtype=torch.float64))
        col = (w[:, None] * rgb[s:s + c]).sum(0)
        op = w.sum()
        if bg is not None:
            col = col + (1 - op) * bg[r]
        outs.append(torch.cat([col, op[None], (w * mid).sum()[None]]))
    return torch.stack(outs)


def test_render_bwd_matches_autograd_of_independent_formulation():
    import torch
    info, t0, t1, sig, rgb, g = _random_packed(61)
    n = info.shape[0]
    bg = g.random((n, 3)).astype(np.float32)
    grads = g.standard_normal((n, 5)).astype(np.float32)
    sig_t = torch.tensor(sig, dtype=torch.float64, requires_grad=True)
    rgb_t = torch.tensor(rgb, dtype=torch.float64, requires_grad=True)
    out = _torch_render(info, t0, t1, sig_t, rgb_t, torch.tensor(bg, dtype=torch.float64))
    (out * torch.tensor(grads, dtype=torch.float64)).sum().backward()
    ds, dr = oracle.render_bwd(info, t0, t1, sig, rgb, grads[:, :3], grads[:, 3], grads[:, 4],
                               bg=bg)
    np.testing.assert_allclose(ds, sig_t.grad.numpy(), rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(dr, rgb_t.grad.numpy(), rtol=1e-9, atol=1e-12)


def test_render_bwd_finite_differences():
    info, t0, t1, sig, rgb, g = _random_packed(62, n_rays=6, max_count=12)
    n = info.shape[0]
    gr = g.standard_normal((n, 3))
    gh = g.standard_normal(n)
    gq = g.standard_normal(n)

    def loss(sig64):
        # oracle_render_fwd takes float32 inputs; evaluate the FD in float64 through an
        # independent double loop so the step is not lost to float32 rounding
        tot = 0.0
        for r in range(n):
            s, c = info[r]
            opt = 0.0
            for i in range(s, s + c):
                dl = float(t1[i]) - float(t0[i])
                tau = sig64[i] * dl
                w = math.exp(-opt) * -math.expm1(-tau)
                tot += w * (gr[r] @ rgb[i].astype(np.float64) + gh[r]
                            + gq[r] * 0.5 * (float(t0[i]) + float(t1[i])))
                opt += tau
        return tot

    ds, _ = oracle.render_bwd(info, t0, t1, sig, rgb, gr.astype(np.float32),
                              gh.astype(np.float32), gq.astype(np.float32))
    # the oracle consumed float32 grads: evaluate the FD with those same values
    gr, gh, gq = (x.astype(np.float32).astype(np.float64) for x in (gr, gh, gq))
    base = sig.astype(np.float64)
    for i in range(base.size):
        h = 1e-6 * max(1.0, base[i])
        p, m = base.copy(), base.copy()
        p[i] += h
        m[i] -= h
        fd = (loss(p) - loss(m)) / (2 * h)
        assert ds[i] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_render_bwd_closed_forms():
    # dO/dsigma_k = Delta_k T_final ; dC/dc_k = w_k g ; constant colour: dC/dsigma_k = Delta_k c T_final
    n, L, sig = 50, 1.5, 2.3
    info, t0, t1, s, c = _uniform_ray(n, L, sig, [0.3, 0.6, 0.9])
    fwd = oracle.render_fwd(info, t0, t1, s, c, want_weights=True)
    delta = t1.astype(np.float64) - t0
    Tfin = 1 - fwd["opacity"][0]
    ds, _ = oracle.render_bwd(info, t0, t1, s, c, np.zeros((1, 3), np.float32),
                              np.ones(1, np.float32), None)
    np.testing.assert_allclose(ds, delta * Tfin, rtol=1e-9)
    g = np.array([[1.0, -2.0, 0.5]], np.float32)
    ds2, dr2 = oracle.render_bwd(info, t0, t1, s, c, g)
    np.testing.assert_allclose(dr2, fwd["weights"][:, None] * g.astype(np.float64), rtol=1e-12)
    cg = float(np.dot(c[0].astype(np.float64), g[0].astype(np.float64)))
    np.testing.assert_allclose(ds2, delta * cg * Tfin, rtol=1e-8, atol=1e-14)


def test_weights_bwd_is_render_bwd_with_per_sample_cotangent():
    info, t0, t1, sig, rgb, g = _random_packed(63)
    # v_i = g.c_i  for all samples of a ray reproduces render_bwd with that g
    n = info.shape[0]
    gr = g.standard_normal((n, 3)).astype(np.float32)
    rid = np.repeat(np.arange(n), info[:, 1])
    gw = (rgb.astype(np.float64) * gr[rid].astype(np.float64)).sum(1).astype(np.float32)
    ds_w = oracle.weights_bwd(info, t0, t1, sig, gw)
    import torch
    sig_t = torch.tensor(sig, dtype=torch.float64, requires_grad=True)
    # autograd of sum_i w_i gw_i on the independent formulation
    loss = 0
    for r in range(n):
        s, c = int(info[r, 0]), int(info[r, 1])
        delta = torch.tensor(t1[s:s + c], dtype=torch.float64) - torch.tensor(
            t0[s:s + c], dtype=torch.float64)
        tau = sig_t[s:s + c] * delta
        w = torch.exp(-(torch.cumsum(tau, 0) - tau)) * (1 - torch.exp(-tau))
        loss = loss + (w * torch.tensor(gw[s:s + c], dtype=torch.float64)).sum()
    loss.backward()
    np.testing.assert_allclose(ds_w, sig_t.grad.numpy(), rtol=1e-9, atol=1e-12)


# ----------------------------------------------------------------------------
# packed table and repack (Section 4.2, "Packed Tensor"; "No Gradient Filtering")
# ----------------------------------------------------------------------------
def test_exclusive_scan_hand_case():
    info, total = oracle.exclusive_scan(np.array([3, 0, 2, 0, 5], np.int32))
    assert info.dtype == np.int32 and info.shape == (5, 2)
    assert info.tolist() == [[0, 3], [3, 0], [3, 2], [5, 0], [5, 5]]
    assert total == 10
    info, total = oracle.exclusive_scan(np.zeros(0, np.int32))
    assert info.shape == (0, 2) and total == 0


def test_exclusive_scan_total_past_int32_is_exact_and_rows_saturate():
    # 2^30 + 2^30 + 5 = 2^31 + 5: the total needs 64 bits; row 1 would end at
    # 2^31 and row 2 start there, neither addressable by int32 starts
    counts = np.array([2 ** 30, 2 ** 30, 5, 0], np.int32)
    info, total = oracle.exclusive_scan(counts)
    assert total == 2 ** 31 + 5
    assert info.tolist() == [[0, 2 ** 30], [2 ** 31 - 1, 0], [2 ** 31 - 1, 0], [2 ** 31 - 1, 0]]
    # a row ending exactly at INT32_MAX still fits
    info, total = oracle.exclusive_scan(np.array([2 ** 31 - 2, 1, 1], np.int32))
    assert info.tolist() == [[0, 2 ** 31 - 2], [2 ** 31 - 2, 1], [2 ** 31 - 1, 0]]
    assert total == 2 ** 31


def test_exclusive_scan_brute_force_small():
    g = scenes.rng(21)
    for n in (1, 2, 7, 64, 300):
        c = g.integers(0, 9, n).astype(np.int32)
        info, total = oracle.exclusive_scan(c)
        run = 0
        for r in range(n):
            assert info[r, 0] == run and info[r, 1] == c[r]
            run += int(c[r])
        assert total == run


def test_gather_prefix_hand_case_with_gaps():
    # three rays whose rows leave gaps (samples 4-5 and 9-11 belong to no ray);
    # kept prefixes: none, part of the row, the whole row
    info = np.array([[0, 4], [6, 3], [12, 5]], np.int32)
    t0 = np.arange(17, dtype=np.float32)
    t1 = t0 + np.float32(0.5)
    rid = np.array([0, 0, 0, 0, -1, -1, 1, 1, 1, -1, -1, -1, 2, 2, 2, 2, 2], np.int32)
    kept = np.array([0, 2, 5], np.int32)
    out, o0, o1, orid = oracle.gather_prefix(info, kept, t0, t1, rid)
    assert out.tolist() == [[0, 0], [0, 2], [2, 5]]
    assert o0.tolist() == [6.0, 7.0, 12.0, 13.0, 14.0, 15.0, 16.0]
    assert o1.tolist() == [6.5, 7.5, 12.5, 13.5, 14.5, 15.5, 16.5]
    assert orid.tolist() == [1, 1, 2, 2, 2, 2, 2]


def test_gather_prefix_brute_force_small():
    g = scenes.rng(22)
    n = 40
    counts = g.integers(0, 12, n)
    gaps = g.integers(0, 4, n)
    starts = np.cumsum(gaps + np.concatenate([[0], counts[:-1]]))
    info = np.stack([starts, counts], axis=1).astype(np.int32)
    S = int(starts[-1] + counts[-1] + 3)
    t0 = g.uniform(0, 10, S).astype(np.float32)
    t1 = (t0 + g.uniform(0, 1, S)).astype(np.float32)
    rid = g.integers(0, 1000, S).astype(np.int32)
    kept = np.array([g.integers(0, c + 1) for c in counts], np.int32)
    out, o0, o1, orid = oracle.gather_prefix(info, kept, t0, t1, rid)
    pos = 0
    for r in range(n):
        assert out[r, 0] == pos and out[r, 1] == kept[r]
        for j in range(kept[r]):
            src = starts[r] + j
            assert o0[pos] == t0[src] and o1[pos] == t1[src] and orid[pos] == rid[src]
            pos += 1
    assert pos == o0.shape[0] == o1.shape[0] == orid.shape[0]


# ----------------------------------------------------------------------------
# no-gradient filtering
# ----------------------------------------------------------------------------
def test_transmittance_prefix_constant_density():
    thr = load_golden("constants.json")["transmittance_threshold"]
    counts = np.array([400, 400, 400, 5], np.int32)
    info, S = oracle.exclusive_scan(counts)
    dt = np.float32(0.01)
    t0 = np.concatenate([np.arange(c) * dt for c in counts]).astype(np.float32)
    t1 = (t0 + dt).astype(np.float32)
    sigmas = [0.0, 7.3, 123.0, 1e4]
    sig = np.concatenate([np.full(c, s) for c, s in zip(counts, sigmas)]).astype(np.float32)
    kept, band = oracle.transmittance_prefix(info, t0, t1, sig, thr)
    delta = (t1.astype(np.float64) - t0)
    for r, s in enumerate(sigmas):
        if band[r]:
            continue
        lo, c = info[r]
        # T_i = exp(-sigma * sum_{j<i} Delta_j) >= thr  <=>  i <= ln(1/thr)/(sigma Delta)
        cum = np.concatenate([[0.0], np.cumsum(np.float64(np.float32(s)) * delta[lo:lo + c])])[:-1]
        expect = int(np.sum(cum <= math.log(1 / thr)))
        assert kept[r] == expect
    assert kept[0] == 400  # zero density keeps everything
    assert kept[3] == 1    # the first sample always has T = 1
    tau = 123.0 * 0.01
    assert kept[2] == math.floor(math.log(1e4) / np.float64(np.float32(123.0) * dt)) + 1 or band[2]
    del tau


# ----------------------------------------------------------------------------
# inverse-CDF resampling
# ----------------------------------------------------------------------------
def test_resample_exact_dyadic_histogram():
    # bin masses are multiples of 2^-10 (exact); u_k = (k+1/2)/M gives
    # count_i = ceil(M F_{i+1} - 1/2) - ceil(M F_i - 1/2)
    g = scenes.rng(71)
    nb, M = 16, 64
    for trial in range(20):
        m = g.integers(0, 40, nb).astype(np.float64)
        m[g.integers(0, nb)] += 1
        w = m / 1024.0
        F = np.concatenate([[0], np.cumsum(w)])
        edges = np.linspace(0, 1, nb + 1).astype(np.float32)[None]
        u = ((np.arange(M + 1) + 0.5) / M)[:M].astype(np.float32)
        u = np.concatenate([u, [1.0]]).astype(np.float32)[None]
        out, bins, band = oracle.resample(edges, w.astype(np.float32)[None], M,
                                          oracle.MODE_WEIGHTS, u=u)
        Fn = F[-1]
        Fnorm = F / Fn
        expect = np.ceil(M * Fnorm[1:] - 0.5) - np.ceil(M * Fnorm[:-1] - 0.5)
        got = np.bincount(bins[0, :M], minlength=nb)
        assert np.array_equal(got, expect.astype(int)), trial
        # inside a bin the samples are linear in u
        for k in range(M):
            i = bins[0, k]
            frac = (u[0, k] * Fn - F[i]) / w[i]
            assert out[0, k] == pytest.approx(edges[0, i] + frac * (edges[0, i + 1] - edges[0, i]),
                                              rel=1e-12, abs=1e-12)


def test_resample_uniform_and_zero_mass_fall_back_to_uniform_lattice():
    nb, n_out = 8, 32
    edges = np.linspace(1.0, 3.0, nb + 1).astype(np.float32)[None].repeat(2, 0)
    vals = np.stack([np.full(nb, 2.0), np.zeros(nb)]).astype(np.float32)
    out, _, _ = oracle.resample(edges, vals, n_out, oracle.MODE_WEIGHTS)
    np.testing.assert_allclose(out, np.linspace(1.0, 3.0, n_out + 1)[None].repeat(2, 0),
                               rtol=1e-12)


def test_resample_density_mode_uses_one_minus_transmittance():
    # one opaque bin: F jumps to ~1 inside bin 3; all interior edges land in bin 3
    nb, n_out = 8, 16
    edges = np.linspace(0.0, 8.0, nb + 1).astype(np.float32)[None]
    sig = np.zeros((1, nb), np.float32)
    sig[0, 3] = 50.0
    out, bins, _ = oracle.resample(edges, sig, n_out, oracle.MODE_SIGMA)
    assert np.all(bins[0, :-1] == 3) and bins[0, -1] == nb
    # Eq. 3: F(t) = 1 - exp(-int sigma); inside bin 3 the linear inverse of F
    Fn = -math.expm1(-50.0)
    for k in range(n_out):
        u = k / n_out
        assert out[0, k] == pytest.approx(3.0 + u * Fn / Fn, rel=1e-12)
    assert out[0, -1] == 8.0


def test_occupancy_march_is_inverse_cdf_of_skipping_estimator():
    # Table 1 spatial skipping: p = 1[occ]/n_occ is piecewise constant over the lattice;
    # its inverse CDF at u_k = (k+1/2)/n_occ returns exactly the occupied midpoints
    fld = scenes.blob_field(8)
    bits = scenes.occupancy_bits(fld, 16)
    o, d = scenes.sphere_rays(60, seed=81)
    dt = 0.05
    full = oracle.march(o, d, scenes.pack_bits(np.ones(16 ** 3, bool)), 16, dt0=dt)
    occ = oracle.march(o, d, bits, 16, dt0=dt)
    for r in range(60):
        s, c = full["packed_info"][r]
        so, co = occ["packed_info"][r]
        if co == 0:
            continue
        edges = np.concatenate([full["t0"][s:s + c], full["t1"][s + c - 1:s + c]])
        kept_t0 = set(occ["t0"][so:so + co].tolist())
        mask = np.array([t in kept_t0 for t in full["t0"][s:s + c]], np.float32)
        u = np.concatenate([(np.arange(co) + 0.5) / co, [1.0]]).astype(np.float32)
        out, bins, _ = oracle.resample(edges[None], mask[None], co, oracle.MODE_WEIGHTS,
                                       u=u[None])
        mids = 0.5 * (edges[:-1].astype(np.float64) + edges[1:])
        lattice_idx = np.nonzero(mask)[0]
        assert np.array_equal(bins[0, :co], lattice_idx)
        # u_k was rounded to binary32, which moves t by at most a few 1e-7 within the bin
        np.testing.assert_allclose(out[0, :co], mids[lattice_idx], rtol=0, atol=1e-6 * dt * co)


# ----------------------------------------------------------------------------
# analytic field (stand-in for the user's radiance field)
# ----------------------------------------------------------------------------
def test_field_special_points():
    fld = scenes.BlobField(centres=np.array([[0.2, -0.1, 0.3]]), peak=50.0, width=0.1,
                           A=np.eye(3), b=np.array([0.1, -0.2, 0.3]))
    p = fld.packed_params()
    x = np.array([[0.2, -0.1, 0.3], [0.3, -0.1, 0.3], [0.0, 0.0, 0.0]])
    s, c = oracle.field(x, p)
    assert s[0] == pytest.approx(50.0, rel=1e-15)
    assert s[1] == pytest.approx(50.0 * math.exp(-0.5), rel=1e-12)
    sig = lambda z: 1 / (1 + math.exp(-z))
    np.testing.assert_allclose(c[2], [sig(0.1), sig(-0.2), sig(0.3)], rtol=1e-15)
    np.testing.assert_allclose(c[0], [sig(0.3), sig(-0.3), sig(0.6)], rtol=1e-15)


def test_field_shell_is_opaque_and_grid_is_conservative():
    fld = scenes.blob_field(8, shell=True)
    p = fld.packed_params()
    s, _ = oracle.field(np.array([[10.0, 0, 0], [0, 0, -10.0]]), p)
    assert np.all(s >= fld.shell_peak)
    # every point with sigma > tau lies in an occupied cell of the conservative grid
    res = 32
    bits = scenes.occupancy_bits(fld, res, half_extent=1.5)
    occ = scenes.unpack_bits(bits, res ** 3)
    g = scenes.rng(91)
    x = g.uniform(-1.5, 1.5, (20000, 3))
    s, _ = oracle.field(x, p)
    cell = np.clip(np.floor((x + 1.5) / 3.0 * res).astype(int), 0, res - 1)
    idx = cell[:, 0] + res * (cell[:, 1] + res * cell[:, 2])
    assert np.all(occ[idx[s > 0.01]])


# ----------------------------------------------------------------------------
# occupancy-grid EMA update (Section 3.1, Spatial Skipping)
# ----------------------------------------------------------------------------
def test_grid_points_closed_form_and_inside_cells():
    pts = oracle.grid_points(4, n_levels=2, half_extent0=1.5)
    # level 0 cell (0,0,0): centre -1.5 + 0.5 * 0.75
    np.testing.assert_allclose(pts[0], [-1.125] * 3, rtol=0, atol=1e-15)
    # level 1 cell (3,2,1): h = 3, cell 1.5 -> (-3 + 3.5*1.5, -3 + 2.5*1.5, -3 + 1.5*1.5)
    i = 64 + 3 + 4 * (2 + 4 * 1)
    np.testing.assert_allclose(pts[i], [2.25, 0.75, -0.75], rtol=0, atol=1e-15)
    # jittered points stay in their own cells
    res, L = 8, 3
    u = scenes.rng(60).random((L * res ** 3, 3)).astype(np.float32) * np.float32(0.999)
    p = oracle.grid_points(res, n_levels=L, half_extent0=1.5, u=u)
    for l in range(L):
        h = 1.5 * 2 ** l
        q = p[l * res ** 3:(l + 1) * res ** 3]
        cell = np.floor((q + h) / (2 * h / res)).astype(int)
        i = np.arange(res ** 3)
        assert np.array_equal(cell[:, 0], i % res)
        assert np.array_equal(cell[:, 1], (i // res) % res)
        assert np.array_equal(cell[:, 2], i // res ** 2)


def test_grid_ema_closed_forms():
    g = scenes.rng(61)
    d0 = g.exponential(1.0, 256)
    s = g.exponential(1.0, 256)
    # gamma = 0: the cache becomes the new density; gamma = 1: unchanged
    d, occ = oracle.grid_ema(d0, s, 0.0, 0.5)
    assert np.array_equal(d, s) and np.array_equal(occ, s > 0.5)
    d, occ = oracle.grid_ema(d0, s, 1.0, 0.5)
    assert np.array_equal(d, d0)
    # k updates with a constant density: D_k = s + gamma^k (D_0 - s)
    gamma, d = 0.9, d0.copy()
    for _ in range(25):
        d, _ = oracle.grid_ema(d, s, gamma, 0.5)
    np.testing.assert_allclose(d, s + gamma ** 25 * (d0 - s), rtol=1e-13)


# ----------------------------------------------------------------------------
# combined estimator: the grid's occupied span (Section 4.4, "Combined Sampling")
# ----------------------------------------------------------------------------
def test_span_of_one_occupied_cell_is_its_chord_on_the_lattice():
    # an 8^3 grid with cells (3, 4, 4) and (5, 4, 4) occupied; rays along +x
    # through row (y, z) = (4, 4) enter cell 3 at x = -0.375 and leave cell 5 at
    # x = 0.75.  t = x + 3, lattice a = 1.5, dt = 0.011 (no midpoint on a cell
    # face): the span's ends lie within half a step of the faces.
    res, dt = 8, 0.011
    occ = np.zeros(res ** 3, bool)
    for x in (3, 5):
        occ[x + res * (4 + res * 4)] = True
    yz = -1.5 + 0.375 * np.array([4.3, 4.6])
    o = np.array([[-3.0, yz[0], yz[1]], [-3.0, yz[1], yz[0]], [-3.0, 1.0, 1.0]], np.float32)
    d = np.tile(np.float32([[1, 0, 0]]), (3, 1))
    span, hit = oracle.march_span(o, d, scenes.pack_bits(occ), res, dt0=dt)
    assert hit.tolist() == [1, 1, 0]
    assert span[2].tolist() == [0.0, 0.0]
    for r in range(2):
        assert abs(span[r, 0] - (3.0 - 0.375)) <= 0.5 * dt + 1e-6
        assert abs(span[r, 1] - (3.0 + 0.75)) <= 0.5 * dt + 1e-6
        # both ends sit on the lattice a + k dt (the march's own interval ends)
        k = (span[r, 0] - 1.5) / dt
        assert abs(k - round(k)) < 1e-3


def test_span_of_full_and_empty_grids():
    res = 8
    o, d = scenes.sphere_rays(300, radius=20.0, target_half=2.0, seed=43)
    full = scenes.pack_bits(np.ones(res ** 3, bool))
    span, hit = oracle.march_span(o, d, full, res, dt0=0.02)
    tn, tf = oracle.clip(o, d, BMIN, BMAX)
    inside = tn < tf
    # only rays through the cube hit; every chord longer than a step holds a midpoint
    h = hit.astype(bool)
    assert np.all(h <= inside)
    assert np.all(h[inside & (tf - tn > 0.02 + 1e-5)])
    assert h.sum() > 100
    # full grid: the span starts exactly at the entry, ends within half a step of the exit
    assert np.array_equal(span[h, 0], tn[h])
    assert np.all(span[h, 1] <= tf[h]) and np.all(span[h, 1] > tf[h] - 0.01 - 1e-5)
    span0, hit0 = oracle.march_span(o, d, np.zeros_like(full), res, dt0=0.02)
    assert not hit0.any() and not span0.any()


def test_span_bins_closed_form():
    span = np.array([[1.0, 3.0], [0.5, 0.5], [2.0, 2.75]], np.float32)
    e = oracle.span_bins(span, 4)
    assert e[0].tolist() == [1.0, 1.5, 2.0, 2.5, 3.0]
    assert e[1].tolist() == [0.5] * 5
    assert np.allclose(np.diff(e[2]), 0.1875, rtol=0, atol=1e-15)


# ----------------------------------------------------------------------------
# coarse-to-fine PDF estimator: the merged edge rows
# ----------------------------------------------------------------------------
def test_merge_edges_hand_case_and_invariants():
    a = np.array([[0.0, 2.0, 4.0], [1.0, 1.0, 1.0]], np.float32)
    b = np.array([[1.0, 2.0, 3.0, 5.0], [0.0, 1.0, 2.0, 3.0]], np.float32)
    m = oracle.merge_edges(a, b)
    assert m[0].tolist() == [0.0, 1.0, 2.0, 2.0, 3.0, 4.0, 5.0]
    assert m[1].tolist() == [0.0, 1.0, 1.0, 1.0, 1.0, 2.0, 3.0]
    g = scenes.rng(66)
    a = np.sort(g.integers(0, 50, (100, 33)), 1).astype(np.float32)
    b = np.sort(g.integers(0, 50, (100, 17)), 1).astype(np.float32)
    m = oracle.merge_edges(a, b)
    assert np.all(np.diff(m, axis=1) >= 0)
    for r in range(100):  # same multiset of values
        vals, cnt = np.unique(np.concatenate([a[r], b[r]]), return_counts=True)
        mv, mc = np.unique(m[r], return_counts=True)
        assert np.array_equal(vals, mv) and np.array_equal(cnt, mc)


# ----------------------------------------------------------------------------
# inverse CDF, exponential inside the bin (a density constant per bin)
# ----------------------------------------------------------------------------
def test_resample_exponential_single_bin_is_truncated_exponential_quantile():
    # one bin [a, a + L] of density s: the samples are the quantiles of an
    # exponential distribution truncated to the bin
    a, L, s, n = 1.25, 2.0, float(np.float32(1.7)), 16  # exact in binary32
    out, _, _ = oracle.resample(np.float32([[a, a + L]]), np.float32([[s]]), n,
                                oracle.MODE_SIGMA_EXP)
    Fn = -math.expm1(-s * L)
    ref = [a - math.log1p(-(k / n) * Fn) / s for k in range(n + 1)]
    assert np.allclose(out[0], ref, rtol=0, atol=1e-12)


def test_resample_exponential_inverts_the_piecewise_exponential_cdf():
    g = scenes.rng(68)
    n_rays, nb, n_out = 50, 24, 40
    e = np.cumsum(g.uniform(0.01, 0.2, (n_rays, nb + 1)), 1).astype(np.float32)
    v = (g.exponential(3.0, (n_rays, nb)) * (g.random((n_rays, nb)) < 0.6)).astype(np.float32)
    out, bins, _ = oracle.resample(e, v, n_out, oracle.MODE_SIGMA_EXP)
    e64, v64 = e.astype(np.float64), v.astype(np.float64)
    P = np.concatenate([np.zeros((n_rays, 1)), np.cumsum(v64 * np.diff(e64, axis=1), 1)], 1)
    Fn = -np.expm1(-P[:, -1])
    for r in range(n_rays):
        for k in range(n_out + 1):
            t = out[r, k]
            i = min(np.searchsorted(e64[r], t, side="right") - 1, nb - 1)
            Pt = P[r, i] + v64[r, i] * (t - e64[r, i])  # optical depth up to t
            assert abs(-math.expm1(-Pt) - (k / n_out) * Fn[r]) <= 1e-12, (r, k)


def test_resample_exponential_tends_to_linear_for_thin_bins():
    g = scenes.rng(69)
    e = np.cumsum(g.uniform(0.01, 0.2, (20, 33)), 1).astype(np.float32)
    v = (g.uniform(0.5, 1.5, (20, 32)) * 1e-4).astype(np.float32)  # tau ~ 1e-5 per bin
    lin, _, _ = oracle.resample(e, v, 17, oracle.MODE_SIGMA)
    ex, _, _ = oracle.resample(e, v, 17, oracle.MODE_SIGMA_EXP)
    width = np.diff(e.astype(np.float64), axis=1).max()
    assert np.abs(lin - ex).max() <= 1e-4 * width


def test_disparity_bins_closed_form():
    # a ray along +x from x = -3 through the cube [-1.5, 1.5]^3: chord t in [1.5, 4.5];
    # disparity edges 1/(2/3 + (2/9 - 2/3) k/4) = 1.5, 1.8, 2.25, 3, 4.5
    o = np.float32([[-3.0, 0.1, 0.2], [0.0, 0.0, 0.0], [0.0, 5.0, 0.0]])
    d = np.float32([[1.0, 0.0, 0.0], [0.0, 0.0, 1.0], [0.0, 1.0, 0.0]])
    e = oracle.disparity_bins(o, d, BMIN, BMAX, 4, near=0.05)
    assert np.allclose(e[0], [1.5, 1.8, 2.25, 3.0, 4.5], rtol=0, atol=1e-12)
    # origin inside the cube: from the near plane to the exit at 1.5
    assert e[1, 0] == np.float32(0.05) and abs(e[1, -1] - 1.5) < 1e-12
    assert np.all(np.diff(1.0 / e[1]) < 0) and np.allclose(np.diff(np.diff(1.0 / e[1])), 0)
    # a ray that misses: every edge at the near plane
    assert np.allclose(e[2], np.float32(0.05), rtol=0, atol=0)


# ----------------------------------------------------------------------------
# grid over contracted space
# ----------------------------------------------------------------------------
def contract64(x, scale):
    """Mip-NeRF 360's contraction of x / scale, binary64 (independent of the oracle)."""
    y = np.asarray(x, np.float64) / scale
    r = np.linalg.norm(y, axis=-1, keepdims=True)
    return np.where(r <= 1.0, y, (2.0 - 1.0 / np.maximum(r, 1e-300)) * y / np.maximum(r, 1e-300))


def test_contracted_march_along_an_axis_closed_form():
    # ray from the centre along +x; res 8 over [-2, 2]^3: x-cell 7 holds
    # contracted radii [1.5, 2), i.e. distances t >= 2 scale (2 - 1/t = 1.5)
    res, scale, dt = 8, 1.0, 0.01
    occ = np.zeros(res ** 3, bool)
    occ[7 + res * (4 + res * 4)] = True
    o = np.float32([[0.0, 0.01, 0.01]])
    d = np.float32([[1.0, 0.0, 0.0]])
    kw = dict(n_levels=3, half_extent0=1.5, dt0=dt)
    m = oracle.march(o, d, scenes.pack_bits(occ), res, contract_scale=scale, **kw)
    full = oracle.march(o, d, scenes.pack_bits(np.ones(res ** 3, bool)), res, contract_scale=scale,
                        **kw)
    mid = 0.5 * (full["t0"].astype(np.float64) + full["t1"])
    mk = 0.5 * (m["t0"].astype(np.float64) + m["t1"])
    assert m["total"] > 0 and np.all(mk >= 2.0 - 1e-5)
    assert np.isin(mid[mid >= 2.0 + 1e-5], mk).all()


def test_contracted_march_full_grid_is_the_cascade_lattice():
    res = 8
    o, d = scenes.sphere_rays(200, radius=3.0, target_half=0.5, seed=44)
    kw = dict(n_levels=3, half_extent0=1.5, dt0=0.02)
    full = np.ones(res ** 3, bool)
    c = oracle.march(o, d, scenes.pack_bits(full), res, contract_scale=1.5, **kw)
    q = oracle.march(o, d, np.concatenate([scenes.pack_bits(full)] * 3), res, **kw)
    for k in ("counts", "t0", "t1"):
        assert np.array_equal(c[k], q[k])
    e = oracle.march(o, d, scenes.pack_bits(np.zeros(res ** 3, bool)), res, contract_scale=1.5,
                     **kw)
    assert e["total"] == 0


def test_contracted_march_selects_the_samples_in_occupied_cells():
    # random cells of a 16^3 contracted grid: a sample is kept iff its midpoint,
    # contracted in binary64, lies in an occupied cell (up to 1e-5 of a face)
    res, scale = 16, 1.5
    g = scenes.rng(45)
    occ = g.random(res ** 3) < 0.3
    o, d = scenes.sphere_rays(300, radius=3.0, target_half=1.0, seed=46)
    kw = dict(n_levels=4, half_extent0=1.5, dt0=0.03, contract_scale=scale)
    full = oracle.march(o, d, scenes.pack_bits(np.ones(res ** 3, bool)), res, want_level=True,
                        **kw)
    kept = oracle.march(o, d, scenes.pack_bits(occ), res, **kw)
    rid = full["ray_id"]
    # the lattice midpoint t0 + dt_l / 2 (the last interval of a segment is cut
    # at the segment end, so (t0 + t1) / 2 is not its test point)
    tm = full["t0"].astype(np.float64) + 0.5 * 0.03 * 2.0 ** full["level"]
    x = o[rid].astype(np.float64) + tm[:, None] * d[rid].astype(np.float64)
    u = (contract64(x, scale) + 2.0) * (res / 4.0)
    cell = np.clip(np.floor(u), 0, res - 1).astype(np.int64)
    near_face = (np.abs(u - np.round(u)) < 1e-4).any(axis=1)
    want = occ[cell[:, 0] + res * (cell[:, 1] + res * cell[:, 2])]
    key = lambda r, t: r.astype(np.int64) * (1 << 40) + np.round(t * 1e6).astype(np.int64)
    got = np.isin(key(rid, full["t0"]), key(kept["ray_id"], kept["t0"]))
    assert kept["total"] > 100
    assert np.array_equal(got[~near_face], want[~near_face])


def test_contracted_cell_points_map_back_into_their_cells():
    res, scale = 16, 1.5
    u = scenes.rng(47).random((res ** 3, 3)).astype(np.float32) * np.float32(0.98) + np.float32(0.01)
    for uu in (None, u):
        p = oracle.grid_points_contracted(res, scale, center=(0.25, -0.125, 0.375), u=uu)
        idx = np.arange(res ** 3)
        cell = np.stack([idx % res, (idx // res) % res, idx // (res * res)], 1)
        zc = -2.0 + (cell + (0.5 if uu is None else uu.astype(np.float64))) * (4.0 / res)
        inside = np.linalg.norm(zc, axis=1) < 2.0 - 1e-9
        back = contract64(p - np.array([0.25, -0.125, 0.375]), scale)
        assert np.allclose(back[inside], zc[inside], rtol=0, atol=1e-9)
        assert np.all(np.linalg.norm(p[~inside], axis=1) > 1e3)


def test_grid_bricks_hand_cases():
    """Brick occupancy (the coarse level the march skips empty space with),
    hand-derived on a 16^3 grid of 2^3 bricks: one cell at the far corner of
    brick (0,0,0), then one cell at the near corner of brick (1,0,0).  A plain
    bit marks the brick holding the cell; a block bit marks every brick whose
    2x2x2 block (itself and its +x, +y, +z neighbours) holds it."""
    res = 16
    idx = lambda x, y, z: x + res * (y + res * z)
    bidx = lambda x, y, z: x + 2 * (y + 2 * z)
    occ = np.zeros(res ** 3, bool)
    occ[idx(7, 7, 7)] = True
    b = oracle.grid_bricks(scenes.pack_bits(occ), res)
    assert b.shape == (1, 2, 8)
    assert np.flatnonzero(b[0, 0]).tolist() == [bidx(0, 0, 0)]
    assert np.flatnonzero(b[0, 1]).tolist() == [bidx(0, 0, 0)]
    occ[:] = False
    occ[idx(8, 0, 0)] = True
    b = oracle.grid_bricks(scenes.pack_bits(occ), res)
    assert np.flatnonzero(b[0, 0]).tolist() == [bidx(1, 0, 0)]
    assert sorted(np.flatnonzero(b[0, 1]).tolist()) == [bidx(0, 0, 0), bidx(1, 0, 0)]
    # a cell of brick (1,1,1) is in the block of all eight bricks; levels are
    # independent; an empty grid has no bit
    occ[:] = False
    occ[idx(15, 9, 12)] = True
    two = np.concatenate([np.zeros(res ** 3, bool), occ])
    b = oracle.grid_bricks(scenes.pack_bits(two), res, n_levels=2)
    assert not b[0].any()
    assert np.flatnonzero(b[1, 0]).tolist() == [bidx(1, 1, 1)]
    assert b[1, 1].all()


def test_grid_bricks_against_brute_force():
    """Each brick bit equals the OR of the cell bits it covers, cell by cell."""
    res = 32
    occ = scenes.unpack_bits(scenes.random_bits(res, 0.002, 11), res ** 3)
    b = oracle.grid_bricks(scenes.pack_bits(occ), res)
    nb = res // 8
    for j in range(nb ** 3):
        bx, by, bz = j % nb, (j // nb) % nb, j // (nb * nb)
        plain = any(occ[x + res * (y + res * z)]
                    for z in range(8 * bz, 8 * bz + 8) for y in range(8 * by, 8 * by + 8)
                    for x in range(8 * bx, 8 * bx + 8))
        assert b[0, 0, j] == plain
    for j in range(nb ** 3):
        bx, by, bz = j % nb, (j // nb) % nb, j // (nb * nb)
        blk = any(b[0, 0, x + nb * (y + nb * z)]
                  for z in range(bz, min(bz + 2, nb)) for y in range(by, min(by + 2, nb))
                  for x in range(bx, min(bx + 2, nb)))
        assert b[0, 1, j] == blk
    assert 0 < b[0, 0].sum() < nb ** 3
