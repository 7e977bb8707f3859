"""The tile raster evaluates each edge function E = a px + b py + c in float64
(a = -dy, b = dx, c = dy xa - dx ya, formed once per triangle) where the
definition (Eq. 1 sampled with the top-left rule, as the oracle computes it)
is the 64-bit integer dx (py - ya) - dy (px - xa).  The two agree exactly when
every product and partial sum is an integer of magnitude below 2^53.  These
tests check that bound over the whole input range the setup admits
(fixed-point coordinates |X|, |Y| < 2^23 from the screen guard |s| < 32768
pixels with 8 sub-pixel bits; sample centres of views up to 8192 pixels) and
check the float64 evaluation against the integer one on random and extreme
triangles.  CPU only."""
import numpy as np

GUARD_FIXED = 32768 * 256          # |X|, |Y| < 2^23
MAX_SIDE = 8192                    # largest view side
SUB = 256


def _exact(xa, ya, xb, yb, px, py):
    return (xb - xa) * (py - ya) - (yb - ya) * (px - xa)


def _plane_f64(xa, ya, xb, yb, px, py):
    a = np.float64(-(yb - ya))
    b = np.float64(xb - xa)
    c = np.float64((yb - ya) * xa - (xb - xa) * ya)
    # the kernel's fma(a, px, fma(b, py, c)); with exact integer operands
    # below 2^53 each product and sum is exact, so the order does not matter
    return a * np.float64(px) + (b * np.float64(py) + c)


def test_bounds_leave_float64_exact():
    lim = GUARD_FIXED - 1
    dmax = 2 * lim                             # |dx|, |dy|
    pmax = MAX_SIDE * SUB + SUB // 2           # largest sample centre
    assert dmax * pmax < 2 ** 46
    cmax = 2 * dmax * lim                      # |dy xa - dx ya|
    assert cmax < 2 ** 48
    assert 2 * dmax * pmax + cmax < 2 ** 53


def test_plane_form_matches_integer_edge_function():
    rng = np.random.default_rng(7)
    lim = GUARD_FIXED - 1
    cases = []
    for _ in range(20000):
        xa, ya, xb, yb = (int(v) for v in rng.integers(-lim, lim + 1, 4))
        px = int(rng.integers(0, MAX_SIDE)) * SUB + SUB // 2
        py = int(rng.integers(0, MAX_SIDE)) * SUB + SUB // 2
        cases.append((xa, ya, xb, yb, px, py))
    # extremes: corners of the admissible range and the farthest sample
    far = (MAX_SIDE - 1) * SUB + SUB // 2
    for xa in (-lim, lim):
        for ya in (-lim, lim):
            for xb in (-lim, lim):
                for yb in (-lim, lim):
                    for px in (SUB // 2, far):
                        for py in (SUB // 2, far):
                            cases.append((xa, ya, xb, yb, px, py))
    for xa, ya, xb, yb, px, py in cases:
        e = _exact(xa, ya, xb, yb, px, py)
        f = _plane_f64(xa, ya, xb, yb, px, py)
        assert f == float(e) and int(f) == e, (xa, ya, xb, yb, px, py)


def test_sign_and_zero_preserved_on_shared_edges():
    """Samples exactly on an edge (E = 0) decide the top-left rule: the
    float64 form must return exactly zero there."""
    rng = np.random.default_rng(8)
    for _ in range(2000):
        # an edge through two sample centres, so that samples on the line exist
        i0, j0 = (int(v) for v in rng.integers(0, MAX_SIDE, 2))
        di, dj = (int(v) for v in rng.integers(-64, 65, 2))
        if di == 0 and dj == 0:
            continue
        xa, ya = i0 * SUB + SUB // 2, j0 * SUB + SUB // 2
        xb, yb = xa + di * SUB, ya + dj * SUB
        t = int(rng.integers(-3, 4))
        px, py = xa + t * di * SUB, ya + t * dj * SUB
        assert _exact(xa, ya, xb, yb, px, py) == 0
        assert _plane_f64(xa, ya, xb, yb, px, py) == 0.0
