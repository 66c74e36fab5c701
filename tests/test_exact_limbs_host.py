"""Host check of the exact limb split used by the 0/1 walks' integer products.

The device computes, for integers x and g with |x|, |g| < 2^51 (so |x g| < 2^102):
h = fl(x g), l = x g - h (an fma), q = fl(h + 1.5*2^103), and the binned low
limb y = fl(fl(h + fl(K - q)) + l) with K = 1.5*2^103 + 1.5*2^52.  The claims
are that every one of these operations is exact, that bits(y) - bits(1.5*2^52)
equals x g - (q - 1.5*2^103) in [-2^51, 2^51], and that (bits(q) -
bits(1.5*2^103)) * 2^51 + that low limb is x g.  IEEE double arithmetic in
numpy rounds like the VALU, so the identities are checked here with Python
integers as the reference.
"""
import numpy as np

C = 1.5 * 2.0 ** 103
M52 = 1.5 * 2.0 ** 52
K = C + M52


def bits(x: float) -> int:
    return int(np.array([x], dtype=np.float64).view(np.int64)[0])


def split(x: int, g: int):
    h = float(np.float64(x) * np.float64(g))
    l_exact = x * g - int(h)
    l = float(l_exact)
    assert int(l) == l_exact  # the fma residual is a double
    q = float(np.float64(h) + np.float64(C))
    t = float(np.float64(K) - np.float64(q))
    y0 = float(np.float64(h) + np.float64(t))
    y = float(np.float64(y0) + np.float64(l))
    return h, l, q, t, y0, y


def samples():
    r = np.random.default_rng(20190413)
    lim = (1 << 51) - 1
    out = [(lim, lim), (-lim, lim), (lim, -lim), (1, 1), (0, 5), (lim, 1), (3, 1 << 50),
           ((1 << 50) + 1, (1 << 51) - 3), (-(1 << 50) - 7, (1 << 50) + 9)]
    for bits_x in (10, 30, 45, 50, 51):
        for bits_g in (10, 30, 45, 50, 51):
            for _ in range(40):
                x = int(r.integers(-(1 << bits_x) + 1, 1 << bits_x))
                g = int(r.integers(-(1 << bits_g) + 1, 1 << bits_g))
                out.append((x, g))
    return out


def test_low_limb_with_folded_offset_is_exact():
    for x, g in samples():
        h, l, q, t, y0, y = split(x, g)
        hr = int(q) - int(C)
        assert hr % (1 << 51) == 0, (x, g)
        assert int(t) == int(M52) - hr, (x, g)  # K - q is exact
        assert int(y0) == int(h) - hr + int(M52), (x, g)  # h + (K - q) is exact
        low = x * g - hr
        assert abs(low) <= 1 << 51, (x, g)
        assert int(y) == low + int(M52), (x, g)  # + l is exact
        assert bits(y) - bits(M52) == low, (x, g)
        assert (bits(q) - bits(C)) * (1 << 51) + low == x * g, (x, g)


def test_folded_constant_is_exact():
    assert K - C == M52 and int(K) == int(C) + int(M52)
