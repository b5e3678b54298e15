"""Index maps of the device code, restated and checked on the CPU.

- The current fold: each tile's current block covers its own cells plus one
  guard column/row below and two above, with periodic wrap; a cell's folded
  current is the sum of the block entries of every tile whose block covers it.
  The device code (`fold_s_body`, `fold_cell` in pic_kernels.hip) finds those
  entries by index arithmetic over the 3 x 3 neighbouring tiles, with a fast
  path for full-height tiles at least 3 columns wide.  Both are compared, cell
  by cell over many grid shapes, with coverage taken from its definition: all
  (tile, block entry) pairs that land on the cell.
- The streaming field kernels' strips own every cell exactly once.
- The particle hand-off delivers every leaver to exactly one tile.
- The push's work order (`k_order`, `order_block`): a stable counting sort of
  the items into load buckets, heaviest first, dealt to the XCDs in chunks;
  every item gets exactly one block.
"""
import itertools
import random

import pytest

TX = TY = 16


def tiles(n):
    return [(a, min(TX, n - TX * a)) for a in range((n + TX - 1) // TX)]


def brute(nxs, ny, gx, gy):
    """Every (tile x, block column, tile y, block row) whose entry is the cell."""
    xs = [(a, px + 1) for a, w in tiles(nxs) for px in range(-1, w + 2)
          if (TX * a + px) % nxs == gx]
    ys = [(b, py + 1) for b, h in tiles(ny) for py in range(-1, h + 2)
          if (TY * b + py) % ny == gy]
    return sorted((a, cx, b, cy) for (a, cx), (b, cy) in itertools.product(xs, ys))


def reach(n, size):
    """Tiles searched on each side along an axis of n cells: one, or two when
    the last tile is one cell wide (the guards of the tile before it then
    reach over it)."""
    return 2 if n % size == 1 else 1


def span_off(l, o, t, n, size):
    """Offset of cell l of tile t within the block of tile t + o (periodic)."""
    nt = (n + size - 1) // size
    ext = lambda a: min(size, n - size * a)
    p = l
    if o < 0:
        for k in range(1, -o + 1):
            p += ext((t - k) % nt)
    else:
        for k in range(o):
            p -= ext((t + k) % nt)
    return p


def general(nxs, ny, gx, gy, rx=None, ry=None):
    """The neighbour search over (2 reach + 1)^2 tiles, in its (oy, ox) order."""
    ntx, nty = (nxs + TX - 1) // TX, (ny + TY - 1) // TY
    rx = reach(nxs, TX) if rx is None else rx
    ry = reach(ny, TY) if ry is None else ry
    tx, ty = gx // TX, gy // TY
    lx, ly = gx - TX * tx, gy - TY * ty
    out = []
    for oy in range(-ry, ry + 1):
        tyn = (ty + oy) % nty
        hn = min(TY, ny - TY * tyn)
        py = span_off(ly, oy, ty, ny, TY)
        if py < -1 or py >= hn + 2:
            continue
        for ox in range(-rx, rx + 1):
            txn = (tx + ox) % ntx
            wn = min(TX, nxs - TX * txn)
            px = span_off(lx, ox, tx, nxs, TX)
            if px < -1 or px >= wn + 2:
                continue
            out.append((txn, px + 1, tyn, py + 1))
    return out


def fast(nxs, ny, gx, gy):
    """The path for a full-height tile at least 3 columns wide on a grid with
    no one-cell tile (None otherwise)."""
    ntx, nty = (nxs + TX - 1) // TX, (ny + TY - 1) // TY
    tx, ty = gx // TX, gy // TY
    lx, ly = gx - TX * tx, gy - TY * ty
    w, h = min(TX, nxs - TX * tx), min(TY, ny - TY * ty)
    if not (reach(nxs, TX) == 1 and reach(ny, TY) == 1 and h == TY and w >= 3):
        return None
    txl, txr = (tx - 1) % ntx, (tx + 1) % ntx
    wl = min(TX, nxs - TX * txl)
    xo = -1 if lx < 2 else (1 if lx == w - 1 else 0)
    txn = txl if xo < 0 else (txr if xo > 0 else tx)
    cxo, cxn = lx + 1, (lx + wl + 1 if xo < 0 else (0 if xo > 0 else lx + 1))

    def level(tyn, row):
        if xo < 0:
            return [(txn, cxn, tyn, row), (tx, cxo, tyn, row)]
        if xo > 0:
            return [(tx, cxo, tyn, row), (txn, cxn, tyn, row)]
        return [(tx, cxo, tyn, row)]

    out = []
    if ly < 2:
        tyl = (ty - 1) % nty
        out += level(tyl, ly + min(TY, ny - TY * tyl) + 1)
    out += level(ty, ly + 1)
    if ly == TY - 1:
        out += level((ty + 1) % nty, 0)
    return out


def shapes():
    rng = random.Random(7)
    yield from [(4, 4), (2, 2), (3, 70), (18, 20), (34, 18), (32, 32), (16, 16), (48, 34)]
    # one-cell last tiles along x, y or both, and two-tile grids that wrap
    yield from [(17, 20), (33, 16), (49, 33), (20, 17), (17, 17), (65, 49), (33, 2), (2, 33)]
    for _ in range(40):
        yield rng.randrange(2, 70), rng.randrange(2, 70)
    # moving-window storage widths are multiples of 16
    yield from [(32, 20), (64, 9), (80, 34)]


@pytest.mark.parametrize("nxs,ny", list(shapes()))
def test_fold_selects_exactly_the_covering_block_entries(nxs, ny):
    for gy in range(ny):
        for gx in range(nxs):
            g = general(nxs, ny, gx, gy)
            assert sorted(g) == brute(nxs, ny, gx, gy), (gx, gy)
            f = fast(nxs, ny, gx, gy)
            if f is not None:
                # the same entries, added in the same order
                assert f == g, (gx, gy)


def test_a_one_cell_tile_needs_the_wider_search():
    # why a grid that leaves a one-cell tile searches two tiles each way: the
    # guard columns of the tile two to the left reach over the one-cell tile,
    # beyond a 3 x 3 neighbour search
    for nxs, ny in ((33, 16), (16, 33)):
        misses = [(gx, gy) for gy in range(ny) for gx in range(nxs)
                  if sorted(general(nxs, ny, gx, gy, rx=1, ry=1)) != brute(nxs, ny, gx, gy)]
        assert misses


# ---------------------------------------------------------------------------
# the streaming field kernels' work split: strips of columns by rows
# ---------------------------------------------------------------------------
YS_S = 6


def strip_w(rf):
    return 63 - 2 * max(1, rf)


@pytest.mark.parametrize("rf", [0, 1, 2, 3, 4])
def test_yee_strips_own_every_cell_exactly_once(rf):
    # a wavefront of 64 lanes holds columns c0 - P .. c0 + 63 - P and owns
    # lanes P .. P + W - 1 (P = max(1, rf)); the rf filter passes leave lanes
    # rf .. 63 - rf exact, the Yee halo is one lane below and two above
    P, W = max(1, rf), strip_w(rf)
    assert P >= rf and P + W <= 64 - rf and P - 1 >= 0 and P + W + 1 <= 63
    rng = random.Random(rf)
    for nxs, ny in [(2, 2), (3, 70), (61, 7), (62, 12), (64, 64), (130, 40)] + \
            [(rng.randrange(2, 300), rng.randrange(2, 50)) for _ in range(20)]:
        ncg = (nxs + W - 1) // W
        units = ncg * ((ny + YS_S - 1) // YS_S)
        seen = {}
        for blk in range(units):
            cg, r0 = blk % ncg, (blk // ncg) * YS_S
            nr = min(YS_S, ny - r0)
            for L in range(64):
                cx = cg * W + L - P
                if not (P <= L < P + W and cx < nxs):
                    continue
                for m in range(nr):
                    key = (cx, r0 + m)
                    assert key not in seen, (nxs, ny, key)
                    seen[key] = blk
        assert len(seen) == nxs * ny, (nxs, ny)


def test_the_model_uses_the_device_constants():
    import os
    import re
    h = open(os.path.join(os.path.dirname(__file__), "..", "paper_2106_12485_amd", "csrc",
                          "pic_dev.h")).read()
    assert re.search(r"constexpr int TX = 16\b", h) and re.search(r"constexpr int TY = 16\b", h)
    assert re.search(r"constexpr int YS_S = %d;" % YS_S, h)
    assert "return 63 - 2 * (rf > 1 ? rf : 1);" in h


# ---------------------------------------------------------------------------
# the particle hand-off: each leaver is picked up by exactly one tile
# ---------------------------------------------------------------------------
def dir_index(dtx, dty):
    k = (dtx + 1) + 3 * (dty + 1)  # 0..8 without the centre 4
    return k if k < 4 else k - 1


def neighbour_slots(t, ntx, nty):
    """(neighbour tile, direction wanted) for the 8 slots of tile t."""
    tx, ty = t % ntx, t // ntx
    out = []
    for k in range(8):
        k9 = k if k < 4 else k + 1
        ox, oy = k9 % 3 - 1, k9 // 3 - 1
        nb = (tx + ox) % ntx + ((ty + oy) % nty) * ntx
        out.append((nb, dir_index(-ox, -oy)))
    return out


@pytest.mark.parametrize("ntx,nty", [(1, 1), (1, 3), (2, 1), (2, 2), (3, 2), (4, 5)])
def test_every_leaver_is_taken_by_exactly_one_tile(ntx, nty):
    # a leaver of tile a stepping by (dtx, dty) (0 along an axis of one tile,
    # which wraps onto itself) is read from a's outbox by the slots of the
    # tile it lands in whose neighbour is a and whose wanted direction is its own
    for a in range(ntx * nty):
        ax, ay = a % ntx, a // ntx
        for dtx, dty in itertools.product((-1, 0, 1), repeat=2):
            if (dtx, dty) == (0, 0) or (ntx == 1 and dtx) or (nty == 1 and dty):
                continue
            dest = (ax + dtx) % ntx + ((ay + dty) % nty) * ntx
            takers = [(b, k) for b in range(ntx * nty)
                      for k, (nb, want) in enumerate(neighbour_slots(b, ntx, nty))
                      if nb == a and want == dir_index(dtx, dty)]
            assert len(takers) == 1 and takers[0][0] == dest, (a, dtx, dty, takers)
    assert sorted(dir_index(x, y) for x, y in itertools.product((-1, 0, 1), repeat=2)
                  if (x, y) != (0, 0)) == list(range(8))


# ---------------------------------------------------------------------------
# the commutative deposit (paper Sec. 3.2): tiles of one checkerboard colour
# add their blocks straight into J in the same launch, so their blocks must
# not share a cell
# ---------------------------------------------------------------------------
def colour_overlaps(nx, ny):
    """Cells reached twice by the blocks of one colour: by two tiles, or by two
    entries of one tile's block (a block wider than the period)."""
    tx_, ty_ = tiles(nx), tiles(ny)
    bad = []
    for colour in range(4):
        seen = {}
        for b, h in ty_:
            if b % 2 != colour >> 1:
                continue
            for a, w in tx_:
                if a % 2 != colour & 1:
                    continue
                for py in range(-1, h + 2):
                    for px in range(-1, w + 2):
                        cell = ((TX * a + px) % nx, (TY * b + py) % ny)
                        if cell in seen:
                            bad.append((colour, cell, seen[cell], (a, b, px, py)))
                        seen[cell] = (a, b, px, py)
    return bad


def test_commutative_colours_never_share_a_cell_where_the_library_accepts_the_grid():
    import ctypes as C
    import os
    from inputs import thermal64
    from paper_2106_12485_amd import build, pic
    lib_path = os.path.join(os.path.dirname(__file__), "..", "paper_2106_12485_amd",
                            "libpic.so")
    if not os.path.exists(lib_path):
        build.build(force=False)
    L = pic.lib()
    accepted = rejected = 0
    for nx in range(2, 100):
        for ny in (2, 3, 18, 19, 32, 34, 35, 50, 64):
            c = pic.make_cfg(thermal64(), deposit="commutative")
            c.nx, c.ny, c.lx, c.ly = nx, ny, 0.1 * nx, 0.1 * ny
            ok = L.pic_mem_bytes(C.byref(c)) > 0
            even = ((nx + 15) // 16) % 2 == 0 and ((ny + 15) // 16) % 2 == 0
            if not even or nx % 16 == 1 or ny % 16 == 1:
                assert not ok, (nx, ny)
                continue
            overl = colour_overlaps(nx, ny)
            # accepted exactly where no two same-colour blocks meet
            assert ok == (not overl), (nx, ny, overl[:3])
            accepted += ok
            rejected += not ok
    assert accepted > 50 and rejected > 5
    # the two grids with a 2-cell last tile that overlapped before they were refused
    assert colour_overlaps(50, 32) and colour_overlaps(18, 20)


# ---------------------------------------------------------------------------
# the push's work order: items sorted into load buckets (stable), dealt to the
# 8 XCDs in chunks of consecutive items (k_order, order_block)
# ---------------------------------------------------------------------------
ORDER_CHUNK = 8


def order_block(p, n, g=ORDER_CHUNK):
    """Block of sorted position p: full rounds of 8 chunks of g positions go to
    the XCDs (block % 8) forwards in even rounds, backwards in odd ones; the
    last, partial round is ranked by (offset in chunk, chunk)."""
    rnd = 8 * g
    full = (n // rnd) * rnd
    if p < full:
        rd, c = p // rnd, (p // g) % 8
        x = 7 - c if rd & 1 else c
        return 8 * (rd * g + p % g) + x
    t, q = n - full, p - full
    x, o = q // g, q % g
    rank = 0
    for c in range((t + g - 1) // g):
        sz = min(g, t - c * g)
        rank += min(sz, o) + (1 if (c < x and sz > o) else 0)
    return full + rank


def load_bucket(w):
    """63 - floor(2 log2(w + 1) + 1/2), clamped to 0..63: heaviest first."""
    import math
    k = math.floor(2.0 * math.log2(w + 1.0) + 0.5)
    return 63 - min(63, max(0, k))


@pytest.mark.parametrize("n", [1, 7, 8, 9, 63, 64, 65, 511, 512, 513, 1024, 2048, 4095,
                               4096, 4100, 16384, 16391])
def test_order_block_is_a_bijection(n):
    assert sorted(order_block(p, n) for p in range(n)) == list(range(n))


def test_order_block_deals_chunks_to_xcds_in_snake_rounds():
    n = 8 * ORDER_CHUNK * 4
    for p in range(n):
        b = order_block(p, n)
        rd, c = p // (8 * ORDER_CHUNK), (p // ORDER_CHUNK) % 8
        assert b % 8 == (7 - c if rd & 1 else c)
        # consecutive positions of a chunk go to consecutive blocks of one XCD
        if p % ORDER_CHUNK:
            assert order_block(p - 1, n) == b - 8


def test_bucket_order_is_heaviest_first_and_stable():
    rng = random.Random(5)
    loads = [rng.choice([0, 3, 4000, 4096, 4200, 8192, 16000, 70000]) for _ in range(3000)]
    n = len(loads)
    keys = [load_bucket(w) for w in loads]
    # the counting sort of k_order: exclusive prefix over buckets, then ranks in
    # item order
    base = [0] * 64
    for k in keys:
        base[k] += 1
    acc = 0
    for k in range(64):
        base[k], acc = acc, acc + base[k]
    pos = []
    for k in keys:
        pos.append(base[k])
        base[k] += 1
    order = [None] * n
    for i, p in enumerate(pos):
        order[order_block(p, n)] = i
    assert sorted(order) == list(range(n))
    by_pos = sorted(range(n), key=lambda i: pos[i])
    # heavier buckets first; within a bucket, item order
    for a, b in zip(by_pos, by_pos[1:]):
        assert keys[a] < keys[b] or (keys[a] == keys[b] and a < b)
    # a load of 2^k sits mid-bucket: +-15% stays in its bucket
    for k in range(6, 20):
        w = 2 ** k
        assert load_bucket(int(w * 0.87)) == load_bucket(w) == load_bucket(int(w * 1.15))


def test_the_order_model_uses_the_device_constants():
    import os
    src = open(os.path.join(os.path.dirname(__file__), "..", "paper_2106_12485_amd", "csrc",
                            "pic_kernels.hip")).read()
    assert "constexpr int ORDER_CHUNK = %d;" % ORDER_CHUNK in src
    assert "floorf(2.0f * __log2f((float)w + 1.0f) + 0.5f)" in src
    assert "return 8 * (rd * G + p % G) + x;" in src
