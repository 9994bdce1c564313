"""CPU model of the two-step kernel's window and ring indexing.

The two-step D2Q9 kernel computes a first step over a window one node wider
than its tile into LDS, then the tile's second step from there.  This model
replays its index logic with numpy on tiny lattices: the window-to-lattice
mapping (wrap or clamp one node past each edge), the halo columns computed
up front, the ring slots each window row goes to (four or three full slots,
or the split rings with the unshifted planes held in a register delay line),
and the neighbour rows and columns the second step reads.  A stand-in
collision (a nonlinear mix of the nine values, bounce-back on walls, fixed
values on the lid) makes any wrong source visible.  Every second-step output
must equal two plain single steps, and no second step may read a ring entry
the first step has not written (NaN sentinels).  The model runs one thread
after another, so it also checks the barrier discipline that makes the
concurrent kernel equal to it: a slot is written again only once a barrier
separates that write from every read of its previous contents (each
iteration has one barrier between its writes and its reads, and the
three-slot ring a second one before its writes).  The GPU tests check the
kernel itself; this checks that its indexing scheme is sound.
"""
import numpy as np
import pytest

CX = [0, 1, 0, -1, 0, 1, -1, -1, 1]
CY = [0, 0, 1, 0, -1, 1, 1, -1, -1]
LID = np.linspace(0.1, 0.9, 9).astype(np.float32)
SHIFTED = [1, 3, 5, 6, 7, 8]


def neighbours(x, y, nx, ny, bc):
    xw, yw = bc == "periodic", bc in ("periodic", "tube")
    xm = x - 1 if x > 0 else (nx - 1 if xw else 0)
    xp = x + 1 if x < nx - 1 else (0 if xw else nx - 1)
    ym = y - 1 if y > 0 else (ny - 1 if yw else 0)
    yp = y + 1 if y < ny - 1 else (0 if yw else ny - 1)
    return xm, xp, ym, yp


def role(x, y, nx, ny, bc):
    if bc == "cavity":
        if y == ny - 1:
            return "lid"
        return "wall" if x in (0, nx - 1) or y == 0 else "fluid"
    if bc == "box":
        return "wall" if x in (0, nx - 1) or y in (0, ny - 1) else "fluid"
    if bc == "tube":
        return "wall" if x in (0, nx - 1) else "fluid"
    return "fluid"


def pull(f, x, y, nx, ny, bc):
    xm, xp, ym, yp = neighbours(x, y, nx, ny, bc)
    cols = {0: x, 1: xm, -1: xp}
    rows = {0: y, 1: ym, -1: yp}
    return np.array([f[q, rows[CY[q]], cols[CX[q]]] for q in range(9)], dtype=np.float32)


def collide(v, r):
    if r == "lid":
        return LID.copy()
    if r == "wall":
        return v[[0, 3, 4, 1, 2, 7, 8, 5, 6]]
    return (v + np.float32(0.1) * np.sin(v.sum() * (np.arange(9) + 1))).astype(np.float32)


def one_step(f, nx, ny, bc):
    g = np.zeros_like(f)
    for y in range(ny):
        for x in range(nx):
            g[:, y, x] = collide(pull(f, x, y, nx, ny, bc), role(x, y, nx, ny, bc))
    return g


def window_map(g, n, wrap):
    if g < 0:
        return n - 1 if wrap else 0
    if g >= n:
        return 0 if (wrap and g == n) else n - 1
    return g


def ring_slot(rs, q, j):
    """(ring, slot, plane) of plane q of window row j."""
    if rs:
        return ("full", j % rs, q)
    if q in (7, 8):
        return ("A", j % 2, q - 7)
    if q in (1, 3):
        return ("B", j % 3, int(q == 3))
    return ("C", j % 4, q - 5)


# Planes the second step reads in the left (x0 - 1) and right (x0 + tw) halo
# columns: those whose velocity points right, and left.
HALO_LEFT = (1, 5, 8)
HALO_RIGHT = (3, 6, 7)


def two_steps(f, nx, ny, bc, bx, h, rs, wave=None):
    """wave: None for tiles of bx columns; else the batch kernel's balanced
    tiles, wave lanes to a wave: the instance's columns spread evenly over
    its ceil(nx / bx) tiles, rounded up to whole waves, with the waves that
    hold no needed column left out of both steps."""
    xw, yw = bc == "periodic", bc in ("periodic", "tube")
    w = bx + 2
    out = np.full_like(f, np.nan)
    tiles_x = (nx + bx - 1) // bx
    if wave is None:
        tw = bx
    else:
        per_tile = -(-nx // tiles_x)  # ceil(nx / tiles_x)
        tw = min(bx, -(-per_tile // wave) * wave)  # rounded up to whole waves
    for ty in range((ny + h - 1) // h):
        for tx in range(tiles_x):
            x0, y0 = tx * tw, ty * h
            hn = min(h, ny - y0)
            # lanes of the waves that take part (all of them for bx-wide tiles)
            lanes = [t for t in range(bx) if wave is None or
                     ((t // wave) * wave < tw and (t // wave) * wave <= nx - x0)]
            halo = np.full((h + 2, 2, 9), np.nan, np.float32)
            for k in range(2 * (hn + 2)):
                side, j = k & 1, k >> 1
                gx = window_map(x0 + tw if side else x0 - 1, nx, xw)
                gy = window_map(y0 - 1 + j, ny, yw)
                halo[j, side] = collide(pull(f, gx, gy, nx, ny, bc), role(gx, gy, nx, ny, bc))
            rings = {"full": np.full((max(rs, 1), 9, w), np.nan, np.float32),
                     "A": np.full((2, 2, w), np.nan, np.float32), "B": np.full((3, 2, w), np.nan, np.float32),
                     "C": np.full((4, 2, w), np.nan, np.float32)}

            def plane(q, j):
                r, sl, p = ring_slot(rs, q, j)
                return rings[r][sl, p]

            # iteration of the last read of each (ring, slot, plane)
            last_read = {}
            gap = 1 if rs == 3 else 2

            def read(q, j, it):
                last_read[ring_slot(rs, q, j)] = it
                return plane(q, j)

            def write(q, j):
                key = ring_slot(rs, q, j)
                assert key not in last_read or j >= last_read[key] + gap, ("slot rewritten too soon", key, j)
                return plane(q, j)

            u0 = np.full(bx, np.nan, np.float32)
            u2a, u2b = u0.copy(), u0.copy()
            for j in range(hn + 2):
                gy = window_map(y0 - 1 + j, ny, yw)
                v = np.full((9, bx), np.nan, np.float32)
                for t in lanes:
                    v[:, t] = collide(pull(f, window_map(x0 + t, nx, xw), gy, nx, ny, bc),
                                      role(window_map(x0 + t, nx, xw), gy, nx, ny, bc))
                written = range(9) if rs else SHIFTED
                for q in written:
                    row = write(q, j)
                    row[1:bx + 1] = v[q]
                    # the kernel keeps a halo column only in the planes that
                    # stream in from its side; the others stay unwritten
                    # (NaN), so a read of one would fail the check below
                    if q in HALO_LEFT:
                        row[0] = halo[j, 0, q]
                    if q in HALO_RIGHT:
                        row[tw + 1] = halo[j, 1, q]
                s0, s2 = u0, u2b
                u0, u2b, u2a = v[0].copy(), u2a, v[2].copy()
                if j < 2:
                    continue
                y = y0 + j - 2
                for t in lanes:
                    x = x0 + t
                    if t >= tw or x >= nx:
                        continue
                    if rs:
                        p0, p2, p4 = read(0, j - 1, j)[t + 1], read(2, j - 2, j)[t + 1], read(4, j, j)[t + 1]
                    else:
                        p0, p2, p4 = s0[t], s2[t], v[4, t]
                    vals = np.array([p0, read(1, j - 1, j)[t], p2, read(3, j - 1, j)[t + 2], p4,
                                     read(5, j - 2, j)[t], read(6, j - 2, j)[t + 2], read(7, j, j)[t + 2],
                                     read(8, j, j)[t]], dtype=np.float32)
                    assert not np.isnan(vals).any(), ("unwritten ring entry read", tx, ty, x, y)
                    out[:, y, x] = collide(vals, role(x, y, nx, ny, bc))
    return out


@pytest.mark.parametrize("rs", [4, 3, 0])
@pytest.mark.parametrize("bc", ["cavity", "box", "tube", "periodic"])
def test_two_step_indexing_equals_two_single_steps(rs, bc):
    rng = np.random.default_rng(7)
    # tiles larger than, equal to and ragged against the lattice; one-row
    # tiles; several tiles per row and column
    for nx, ny, bx, h in [(3, 3, 8, 4), (7, 5, 4, 2), (9, 11, 4, 4), (8, 8, 4, 4), (13, 6, 8, 1), (5, 9, 16, 8)]:
        f = rng.random((9, ny, nx)).astype(np.float32)
        assert np.array_equal(two_steps(f, nx, ny, bc, bx, h, rs), one_step(one_step(f, nx, ny, bc), nx, ny, bc)), \
            (nx, ny, bx, h)


@pytest.mark.parametrize("rs", [3, 0])
@pytest.mark.parametrize("bc", ["cavity", "periodic"])
def test_balanced_batch_tiles_equal_two_single_steps(rs, bc):
    # Widths against 16-lane tiles of 4-lane waves (a 256-thread block of
    # 64-lane waves scaled down): narrower than a tile, a whole number of
    # waves, one column past a tile, two uneven tiles; every needed column is
    # computed by a wave that takes part, and no lane reads a ring entry that
    # a skipped wave would have written.
    rng = np.random.default_rng(8)
    # (20 and 28: the last tile's one-past-the-edge column is the first lane
    # of a wave, which must still take part)
    for nx, ny in [(3, 5), (4, 6), (5, 4), (8, 5), (13, 3), (16, 4), (17, 5), (19, 4), (20, 4), (28, 3), (30, 3),
                   (33, 4)]:
        f = rng.random((9, ny, nx)).astype(np.float32)
        assert np.array_equal(two_steps(f, nx, ny, bc, 16, 2, rs, wave=4),
                              one_step(one_step(f, nx, ny, bc), nx, ny, bc)), (nx, ny)


# --------------------------------------------------------------------------
# D1Q3, up to K steps per launch: the window of each segment, its shrinking
# valid part, and the wall's pull from itself at a lattice end.
# --------------------------------------------------------------------------

def d1q3_collide(f0, fp, fm, wall):
    if wall:
        return f0, fm, fp
    s = f0 + fp + fm
    return (np.float32(f0 + 0.1 * np.sin(s)), np.float32(fp + 0.1 * np.sin(2 * s + fm)),
            np.float32(fm + 0.1 * np.sin(3 * s - fp)))


def d1q3_one_step(f, n, wrap):
    g = np.empty_like(f)
    for x in range(n):
        xm = x - 1 if x > 0 else (n - 1 if wrap else 0)
        xp = x + 1 if x < n - 1 else (0 if wrap else n - 1)
        g[:, x] = d1q3_collide(f[0, x], f[1, xm], f[2, xp], (not wrap) and x in (0, n - 1))
    return g


def d1q3_k_steps(f, n, wrap, seg, kmax, k):
    out = np.full_like(f, np.nan)
    for x0 in range(0, n, seg):
        sn = min(seg, n - x0)
        wl = x0 - kmax if wrap else max(0, x0 - kmax)
        wr = x0 + sn + kmax if wrap else min(n, x0 + sn + kmax)
        L = wr - wl
        lend, rend = (not wrap) and wl == 0, (not wrap) and wr == n
        cur = np.array([f[:, (wl + w) % n] for w in range(L)], dtype=np.float32).T
        for s in range(1, k + 1):
            nxt = np.full_like(cur, np.nan)
            lo, hi = (0 if lend else s), (L if rend else L - s)
            for w in range(lo, hi):
                wm = w if (lend and w == 0) else w - 1
                wp = w if (rend and w == L - 1) else w + 1
                vals = (cur[0, w], cur[1, wm], cur[2, wp])
                assert not np.isnan(vals).any(), ("invalid window node read", x0, s, w)
                nxt[:, w] = d1q3_collide(*vals, (not wrap) and (wl + w) in (0, n - 1))
            cur = nxt
        own0 = x0 - wl
        out[:, x0:x0 + sn] = cur[:, own0:own0 + sn]
    return out


@pytest.mark.parametrize("wrap", [False, True])
def test_d1q3_k_step_indexing_equals_single_steps(wrap):
    rng = np.random.default_rng(11)
    # segments shorter than, equal to and ragged against the lattice; windows
    # wider than a periodic lattice (several wraps); k below and at kmax
    for n, seg, kmax, k in [(3, 4, 2, 2), (10, 4, 3, 3), (10, 4, 3, 1), (17, 8, 5, 4), (5, 2, 6, 6), (40, 16, 4, 4)]:
        f = rng.random((3, n)).astype(np.float32)
        ref = f
        for _ in range(k):
            ref = d1q3_one_step(ref, n, wrap)
        assert np.array_equal(d1q3_k_steps(f, n, wrap, seg, kmax, k), ref), (n, seg, kmax, k)
