"""Bounds the detection kernel's LDS layout relies on (host arithmetic only).

A detection region (a 64-pixel tile plus a filter halo of up to 7 pixels on
each side, clipped at the frame edge) evaluates the background spline piece by
piece along x; its LDS table holds at most 6 pieces per row.  The pieces are
bounded by the mesh centres, so the count follows from the mesh width (at
least 16 pixels, which the library enforces) and the centre rule: piece k
spans [c_{k-1}, c_k) with c_k the centre of mesh k, (a + b - 1) / 2 for a mesh
covering [a, b).
"""

K_NIX_MAX = 6


def _piece_of(p, n, m):
    k0 = p // m
    a = k0 * m
    b = min(a + m, n)
    return k0 + (1 if 2 * p >= a + b - 1 else 0)


def test_region_touches_at_most_six_spline_pieces():
    worst = 0
    for radius in range(0, 8):
        for mw in range(16, 48):
            for width in list(range(1, 260)) + [1000, 1007, 2048, 6144, 6150, 9600]:
                for tx in range((width + 63) // 64):
                    x0 = tx * 64
                    tw = min(64, width - x0)
                    lo = max(0, x0 - radius)
                    hi = min(width - 1, x0 + tw - 1 + radius)
                    worst = max(worst, _piece_of(hi, width, mw) - _piece_of(lo, width, mw) + 1)
    assert worst <= K_NIX_MAX
