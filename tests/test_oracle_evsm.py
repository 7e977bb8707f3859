"""Pins of the oracle's alternative pre-filtered maps: exponentially warped
moments (the pre-warp g = exp of Sec. 3's list of pre-filtered shadow maps)
and the light-bleeding reduction heuristic (supplementary limitations), both
against properties the mathematics fixes and against exact ray casting."""
import math

import numpy as np
import torch

import scenegen as sg
from oracle import pipeline as P
from oracle import raycast


class _L:
    def __init__(self, c=0.0, a=0.0, eps=1e-12):
        self.warp_exponent, self.bleed_reduction, self.min_variance = c, a, eps


def _moments(W2, f, c):
    g = np.exp(c * f) if c > 0 else f
    return (torch.tensor((W2 * g).sum(), dtype=torch.float64), torch.tensor((W2 * g * g).sum(), dtype=torch.float64))


def test_warped_bound_never_below_discrete_pcf():
    """exp is increasing, so the event {depth >= d} is the event
    {exp(c depth) >= exp(c d)}: the one-sided Chebyshev bound on the warped
    moments still bounds the PCF fraction from above (Cantelli), for any
    variance floor."""
    rng = np.random.default_rng(17)
    viol = checked = 0
    for _ in range(6000):
        k = int(rng.choice([3, 5, 7]))
        w = P.filter_taps(str(rng.choice(['box', 'gaussian'])), k, 0.0)
        W2 = np.outer(w, w).ravel()
        f = rng.uniform(0.2, 0.8, k * k)
        if rng.random() < 0.5:
            f[rng.random(k * k) < 0.5] = rng.uniform(0.2, 0.4)
        d = rng.uniform(0.2, 0.8)
        c = float(rng.choice([5.0, 20.0, 40.0]))
        m1, m2 = _moments(W2, f, c)
        v = float(P.lookup_visibility(m1, m2, torch.tensor(d, dtype=torch.float64), _L(c, 0.0, float(rng.choice([1e-12, 1e-5]))))[0])
        pcf = W2[d <= f].sum()
        viol += pcf > v * (1 + 1e-9) + 1e-12
        checked += 1
    assert checked > 5000 and viol == 0


def test_exponential_warp_cuts_two_occluder_light_bleeding():
    """Two occluder layers (half the window at depth 0.2, half at 0.5) over a
    receiver at 0.55: every ray is blocked (PCF 0), yet the plain variance
    bound leaks about a third of the light; the warped bound leaks about
    half a percent (0.25 / (0.25 + (e^2 - 1/2)^2) for c = 40); a bleeding
    reduction of 0.4 removes the plain map's leak."""
    W2 = np.full(16, 1 / 16)
    f = np.array([0.2] * 8 + [0.5] * 8)
    d = torch.tensor(0.55, dtype=torch.float64)
    v_plain = float(P.lookup_visibility(*_moments(W2, f, 0.0), d, _L(0.0))[0])
    v_exp = float(P.lookup_visibility(*_moments(W2, f, 40.0), d, _L(40.0))[0])
    assert abs(v_plain - 0.0225 / (0.0225 + 0.04)) < 1e-12
    assert abs(v_exp - 0.25 / (0.25 + (math.e ** 2 - 0.5) ** 2)) < 1e-6
    assert v_exp < v_plain / 50
    assert float(P.lookup_visibility(*_moments(W2, f, 0.0), d, _L(0.0, 0.4))[0]) == 0.0


def test_bleeding_reduction_keeps_lit_and_order():
    """The reduction maps [a, 1] onto [0, 1] increasingly and everything
    below a to 0: fully lit stays lit, and zero amount changes nothing."""
    rng = np.random.default_rng(3)
    m1 = torch.as_tensor(rng.uniform(0.1, 0.9, 2000))
    m2 = m1 ** 2 + torch.as_tensor(rng.uniform(0, 0.01, 2000))
    d = torch.as_tensor(rng.uniform(0.0, 1.0, 2000))
    v0 = P.lookup_visibility(m1, m2, d, _L(0.0, 0.0, 1e-5))[0]
    assert torch.equal(v0, P.chebyshev(m1, m2, d, 1e-5))
    for a in (0.1, 0.3, 0.6):
        va = P.lookup_visibility(m1, m2, d, _L(0.0, a, 1e-5))[0]
        assert torch.all(va[v0 == 1] == 1)
        assert torch.all(va[v0 <= a] == 0)
        o = torch.argsort(v0)
        assert torch.all(torch.diff(va[o]) >= 0)
        assert torch.all(va <= v0 + 1e-15)


def _hard(cfg, c):
    b = sg.config0() if cfg == 0 else sg.config1()
    for L in b.lights:
        L.k = 1
        L.antialias = False
        L.min_variance = 1e-12
        L.warp_exponent = c
    return b


def test_exponential_maps_store_the_warped_depth():
    """The warped maps hold exp(c z) and exp(2 c z) of the plain maps' z,
    texel by texel, background (exp(c), exp(2c)) included."""
    c = 30.0
    out = []
    for cc in (0.0, c):
        b = _hard(1, cc)
        base, poses, lp, alb = P.scene_leaves(b, requires_grad=False)
        out.append(P.render(b, P.world_vertices(b, base, poses), lp, alb)['lights'][0]['F0'].numpy())
    z = out[0][0]
    assert np.allclose(out[1][0], np.exp(c * z), rtol=1e-13, atol=0)
    assert np.allclose(out[1][1], np.exp(2 * c * z), rtol=1e-13, atol=0)
    assert np.any(z == 1.0) and np.any(z < 1.0)


def test_exponential_hard_shadow_limit_equals_ray_casting():
    """k = 1, no smoothing, tiny floor: the warped test exp(c d) <= exp(c f)
    is the binary shadow-map test of Eq. (2) and must agree with exact ray
    casting where the shadow-map footprint stays on one triangle."""
    from test_oracle_shading import test_hard_shadow_limit_equals_ray_casting as plain
    import test_oracle_shading as T
    orig = T.hard_shadow_batch
    try:
        T.hard_shadow_batch = lambda cfg: _hard(cfg, 40.0)
        plain(0)
        plain(1)
    finally:
        T.hard_shadow_batch = orig
