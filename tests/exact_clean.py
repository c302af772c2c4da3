"""Exact rational Hogbom CLEAN for tiny inputs (a pin for the oracle).

Written independently of the C oracle: Python ``Fraction`` arithmetic, no
rounding anywhere, images as dicts keyed by (y, x).  It follows the textbook
definition of a minor iteration (find the largest |r|, lowest row-major index
on a tie; component = gain * value; subtract component * PSF centred on the
peak), and the tiled form with feedback, where a tile cleans only its own
pixels and, at the end of each round, every component found in the round has
its PSF subtracted from all pixels outside its tile.  A round ends after the
interval or, with a flux level, when the tile's peak falls below that fraction
of the largest tile peak at the round's start.  In exact arithmetic that
equals subtracting the cross-coupling images (component image convolved with
the PSF), so aggregation order and rounding do not enter.
"""
from fractions import Fraction


def to_frac_image(a):
    ny, nx = a.shape
    return {(y, x): Fraction(float(a[y, x])) for y in range(ny) for x in range(nx)}


def peak(r, pixels):
    """(position, value, margin): lowest row-major index among the largest |r|;
    margin is the gap in |r| to the best pixel at any other position."""
    best = None
    for q in sorted(pixels):
        if best is None or abs(r[q]) > abs(r[best]):
            best = q
    others = [abs(r[q]) for q in pixels if q != best]
    margin = abs(r[best]) - max(others) if others else abs(r[best])
    return best, r[best], margin


def subtract(r, pixels, p, c, psf, cy, cx):
    py, px = p
    for (y, x) in pixels:
        r[(y, x)] -= c * psf[(y - py + cy, x - px + cx)]


def hogbom(dirty, psf, gain, threshold, max_iter):
    ny, nx = dirty.shape
    r = to_frac_image(dirty)
    P = to_frac_image(psf)
    cy, cx = psf.shape[0] // 2, psf.shape[1] // 2
    g = Fraction(gain)
    thr = Fraction(threshold)
    pixels = list(r.keys())
    comps, margins = [], []
    while True:
        p, v, m = peak(r, pixels)
        if len(comps) == max_iter or abs(v) < thr:
            break
        c = g * v
        comps.append((p[0] * nx + p[1], c))
        margins.append(m)
        subtract(r, pixels, p, c, P, cy, cx)
    return r, comps, margins


def tile_pixels(ny, nx, ty, tx, t):
    i, j = divmod(t, tx)
    y0, y1 = i * ny // ty, (i + 1) * ny // ty
    x0, x1 = j * nx // tx, (j + 1) * nx // tx
    return [(y, x) for y in range(y0, y1) for x in range(x0, x1)]


def tiled(dirty, psf, tiles, interval, gain, threshold, max_iter, level=0.0):
    ny, nx = dirty.shape
    ty, tx = tiles
    r = to_frac_image(dirty)
    P = to_frac_image(psf)
    cy, cx = psf.shape[0] // 2, psf.shape[1] // 2
    g = Fraction(gain)
    thr = Fraction(threshold)
    T = ty * tx
    tpix = [tile_pixels(ny, nx, ty, tx, t) for t in range(T)]
    all_pix = list(r.keys())
    comps, margins, rounds = [], [], 0
    lev_frac = Fraction(level)
    while True:
        # a tile takes part at or above the threshold and at or above the round's
        # flux level (a fraction of the largest tile peak at the round's start)
        tpk = [abs(peak(r, tpix[t])[1]) for t in range(T)]
        lev = lev_frac * max(tpk)
        active = [tpk[t] >= thr and tpk[t] >= lev for t in range(T)]
        if len(comps) == max_iter or not any(active):
            break
        rem, na = max_iter - len(comps), sum(active)
        budget, rank = [], 0
        for t in range(T):
            if not active[t]:
                budget.append(0)
                continue
            budget.append(interval if rem >= na * interval else rem // na + (1 if rank < rem % na else 0))
            rank += 1
        found = []
        for t in range(T):
            for _ in range(budget[t]):
                p, v, m = peak(r, tpix[t])
                if abs(v) < thr or abs(v) < lev:
                    break
                c = g * v
                found.append((t, p, c))
                margins.append(m)
                subtract(r, tpix[t], p, c, P, cy, cx)
        own = [set(tp) for tp in tpix]
        for (t, p, c) in found:
            outside = [q for q in all_pix if q not in own[t]]
            subtract(r, outside, p, c, P, cy, cx)
        comps.extend((p[0] * nx + p[1], c) for (t, p, c) in found)
        rounds += 1
    return r, comps, margins, rounds
