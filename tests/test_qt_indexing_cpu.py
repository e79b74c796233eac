"""CPU replay of the chunked quarter-turn backprojector's window coordinates.

The kernel stages, per (tile, angle pair), a window of WP bins that starts one bin
below the smallest ray coordinate of the tile, and reads bins j and (through the
staged differences) j + 1 at j = trunc(u) of each pixel's FP32 local coordinate.
This file restates in NumPy the host's window bound and pitch choice and the
kernel's FP64 window origins and FP32 coordinate arithmetic (fused multiply-adds
rounded once), and asserts that every bin a pixel reads was staged: 0 <= j and
j <= WP - 2 (the last bin of a window has no staged difference).  It covers the
GPU test geometries and the benchmark workloads (512^2 / 720 angles / 725 bins,
and the mixed-batch sides 256 ... 1024).  It also replays how the grid and list
kernels hand tiles to workgroups (one per tile, or persistent workgroups taking
per-XCD ranges) and checks that every tile is backprojected exactly once.  No GPU
is involved.
"""
import math

import numpy as np
import pytest

TILE, CHUNKS, ROWS = 16, 16, 4


def f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def fma32(a, b, c):
    """fmaf: the exact a*b + c rounded once to FP32 (the product of two FP32 values is
    exact in FP64, and the sum's rounding to FP64 cannot move it across an FP32
    rounding boundary by more than the checks' margin)."""
    d = lambda x: np.asarray(x, dtype=np.float64)
    return f32(d(a) * d(b) + d(c))


def pitch_for(K, N, dt, angles):
    c = np.cos(angles) / dt
    s = np.sin(angles) / dt
    span = np.max((TILE - 1) * (np.abs(c) + np.abs(s)))
    wl = int(span) + 5
    if wl <= 31:
        return 32
    if wl <= 63:
        return 64
    return 0


def tile_grid(N):
    """Quadrant tiles across and down: the base region is rows [0, N/2) by columns
    [0, (N+1)/2) (a pinwheel piece for odd N)."""
    return ((N + 1) // 2 + TILE - 1) // TILE, (N // 2 + TILE - 1) // TILE


def replay(K, D, N, dt, angles, WP=None):
    """Pitch, and the smallest and largest bin read over every tile, pair and pixel."""
    WP = pitch_for(K, N, dt, angles) if WP is None else WP
    assert WP in (32, 64)
    KH = K // 2
    cd = np.cos(angles[:KH]) / dt
    sd = np.sin(angles[:KH]) / dt
    tiles_x, tiles_y = tile_grid(N)
    hp, cdet = 0.5 * (N - 1), 0.5 * (D - 1)
    c0, r0 = [a.ravel() for a in np.meshgrid(np.arange(tiles_x) * TILE, np.arange(tiles_y) * TILE, indexing="xy")]
    x0 = (c0 - hp)[:, None]
    y0 = (r0 - hp)[:, None]
    uo = x0 * cd + y0 * sd + cdet
    umin = uo + np.minimum(0.0, (TILE - 1) * cd) + np.minimum(0.0, (TILE - 1) * sd)
    vo = x0 * sd - y0 * cd + cdet
    vmin = vo + np.minimum(0.0, (TILE - 1) * sd) + np.minimum(0.0, -(TILE - 1) * cd)
    iu = np.floor(umin).astype(np.int64) - 1
    iv = np.floor(vmin).astype(np.int64) - 1
    bU, bV = f32(uo - iu), f32(vo - iv)
    c32, s32 = f32(cd)[None, :], f32(sd)[None, :]
    lo, hi = np.inf, -np.inf
    for lx in range(TILE):
        for ly0 in range(0, TILE, ROWS):
            u0 = fma32(np.float32(lx), c32, fma32(np.float32(ly0), s32, bU))
            v0 = fma32(np.float32(lx), s32, fma32(np.float32(-ly0), c32, bV))
            for i in range(ROWS):
                u = u0 if i == 0 else fma32(np.float32(i), s32, u0)
                v = v0 if i == 0 else fma32(np.float32(-i), c32, v0)
                assert np.all(u > 0.0) and np.all(v > 0.0), "truncation would not be floor"
                ju = np.trunc(u)
                jv = np.trunc(v)
                lo = min(lo, ju.min(), jv.min())
                hi = max(hi, ju.max(), jv.max())
    return WP, int(lo), int(hi)


def _uniform(K):
    return np.arange(K) * (math.pi / K)


@pytest.mark.parametrize("K,D,N,dt", [
    (2, 3, 2, 1.0), (90, 101, 70, 1.0), (180, 183, 128, 1.0), (40, 75, 50, 0.7), (4, 9, 100, 1.0),
    (720, 725, 512, 1.0), (360, 365, 256, 1.0), (1440, 546, 384, 1.0), (720, 1451, 1024, 1.0),
    (30, 101, 64, 0.36),
    # odd sides: pinwheel quadrants
    (2, 3, 3, 1.0), (90, 101, 71, 1.0), (180, 183, 127, 1.0), (720, 725, 511, 1.0), (40, 75, 49, 0.7),
    (4, 7, 35, 1.3),
])
def test_qt_reads_stay_in_the_staged_window(K, D, N, dt):
    WP, lo, hi = replay(K, D, N, dt, _uniform(K))
    # the window starts one bin below the tile's smallest coordinate, so exact
    # coordinates are >= 1; where that coordinate is an integer (pixel centres on
    # whole offsets, as for odd sides) FP32 rounding can leave it just below 1,
    # and bin 0 (staged) is read
    assert lo >= 0
    assert hi <= WP - 2
    # the host's bound leaves two bins of margin above the largest bin read
    assert hi <= WP - 4


def test_qt_lds_fits_one_workgroup():
    """Static LDS of the two pitches (16 waves x (constants of 64 pairs + B pairs x 4
    planes x WP bins x 16 bytes), plus the chunk sums in a region of their own)
    stays within gfx950's 160 KB."""
    for wp, b in ((32, 2), (64, 1)):
        prm = 64 * 24
        windows = CHUNKS * (prm + b * 4 * wp * 16)
        parts = CHUNKS * 4 * TILE * (TILE + 1) * 4
        assert windows + parts <= 160 * 1024


def test_replay_catches_a_pitch_too_small_for_the_window():
    """The replay has teeth: at dt = 0.7 the window needs the 64-bin pitch; with the
    32-bin one some pixel would read past the staged bins."""
    K, D, N, dt = 40, 75, 50, 0.7
    WP, lo, hi = replay(K, D, N, dt, _uniform(K))
    assert WP == 64 and lo >= 1 and hi <= WP - 4
    _, _, hi32 = replay(K, D, N, dt, _uniform(K), WP=32)
    assert hi32 > 32 - 2


def xcd_logical(b, G):
    """The kernels' block -> logical item map: XCD b % 8 takes a contiguous range."""
    x, slot = b & 7, b >> 3
    per, extra = G >> 3, G & 7
    return x * per + min(x, extra) + slot


def grid_tiles(G, total, persist):
    """Tiles each workgroup of the quarter-turn grid kernel visits, in order (a
    restatement of its start / end / step choice)."""
    out = []
    for b in range(G):
        if not persist or G >= total:
            it = xcd_logical(b, G)
            end, step = it + 1, 1
        elif G % 8 == 0:
            x, per = b & 7, G >> 3
            it = (x * total >> 3) + (b >> 3)
            end, step = (x + 1) * total >> 3, per
        else:
            it, end, step = b, total, G
        seq = []
        while it < end:
            seq.append(it)
            it += step
        out.append(seq)
    return out


def test_xcd_logical_is_a_bijection():
    for G in range(1, 600):
        assert sorted(xcd_logical(b, G) for b in range(G)) == list(range(G))


@pytest.mark.parametrize("cus", [256, 255, 248, 80, 8, 7, 1])
@pytest.mark.parametrize("total", [1, 7, 64, 255, 256, 257, 1000, 256 * 16, 65536 + 3])
def test_grid_kernel_visits_every_tile_once(cus, total):
    """The host launches min(total, CUs) workgroups, persistent when that is fewer
    than the tiles; every tile is then backprojected by exactly one workgroup, and
    with a grid that is a multiple of 8 each XCD's tiles are one contiguous range."""
    G = min(total, cus)
    persist = G < total
    seqs = grid_tiles(G, total, persist)
    flat = sorted(t for s in seqs for t in s)
    assert flat == list(range(total))
    if persist and G % 8 == 0:
        for x in range(8):
            mine = sorted(t for b in range(x, G, 8) for t in seqs[b])
            assert mine == list(range(x * total >> 3, (x + 1) * total >> 3))


def test_list_kernel_visits_every_tile_once():
    """The list kernels start at xcd_logical(block) and stride by the grid size."""
    for G in (1, 7, 8, 255, 256):
        for total in (0, 1, 5, 256, 1001):
            seen = []
            for b in range(G):
                it = xcd_logical(b, G)
                while it < total:
                    seen.append(it)
                    it += G
            assert sorted(seen) == list(range(total))


def epilogue_writes(N):
    """Image offsets the epilogue writes for every tile of one slice: thread t of
    1024 takes turn t / 256 and tile element t % 256 (rows along tiles for turns 0
    and 2, columns for 1 and 3), writes when its base pixel lies in the base region,
    and for odd N the first tile's wave 0 also writes the centre pixel."""
    tiles_x, tiles_y = tile_grid(N)
    out = []
    for ty_t in range(tiles_y):
        for tx_t in range(tiles_x):
            r0, c0 = ty_t * TILE, tx_t * TILE
            for t in range(1024):
                turn, e = t >> 8, t & 255
                ty = (e % TILE) if (turn & 1) else (e // TILE)
                tx = (e // TILE) if (turn & 1) else (e % TILE)
                r, c = r0 + ty, c0 + tx
                if r < (N >> 1) and c < ((N + 1) >> 1):
                    if turn == 0:
                        o = r * N + c
                    elif turn == 1:
                        o = c * N + (N - 1 - r)
                    elif turn == 2:
                        o = (N - 1 - r) * N + (N - 1 - c)
                    else:
                        o = (N - 1 - c) * N + r
                    out.append(o)
            if (N & 1) and r0 == 0 and c0 == 0:
                out.append((N >> 1) * N + (N >> 1))
    return out


@pytest.mark.parametrize("N", [2, 3, 4, 5, 16, 17, 31, 32, 33, 34, 35, 63, 64, 71, 127, 128, 255])
def test_every_pixel_written_exactly_once(N):
    """The four turns of the base region (a pinwheel piece for odd N) plus, for odd
    N, the centre pixel written by the first tile, cover the N x N image once."""
    writes = epilogue_writes(N)
    assert sorted(writes) == list(range(N * N))


def test_turn_of_a_pixel_keeps_its_ray_coordinate():
    """Turning a pixel by +90 degrees about the centre (x, y) -> (-y, x), as the
    epilogue's index map does for (r, c) -> (c, N-1-r), with its angle turned by
    pi/2 leaves u unchanged: the identity the kernel builds on, for odd N too."""
    rng = np.random.default_rng(7)
    for N in (5, 6, 33):
        h = 0.5 * (N - 1)
        for _ in range(50):
            r, c = int(rng.integers(0, N)), int(rng.integers(0, N))
            th = rng.uniform(0, math.pi)
            x, y = c - h, r - h
            r1, c1 = c, N - 1 - r                     # turned pixel's row and column
            x1, y1 = c1 - h, r1 - h
            u0 = x * math.cos(th) + y * math.sin(th)
            u1 = x1 * math.cos(th + math.pi / 2) + y1 * math.sin(th + math.pi / 2)
            assert abs(u0 - u1) < 1e-9


def fan_turn_writes(N, split=1):
    """Image offsets (and partial planes) the fan-beam quarter-turn kernel writes:
    a 256-thread workgroup per (part, base-region tile), thread (dx, dy) of the
    tile writing its pixel's four turns when the pixel lies in rows [0, N/2) and
    columns [0, (N+1)/2); for odd N the first tile also writes the centre."""
    TF = 16
    tiles_x, tiles_y = ((N + 1) // 2 + TF - 1) // TF, (N // 2 + TF - 1) // TF
    tiles = tiles_x * tiles_y
    out = []
    for b in range(tiles * split):
        g, tile = divmod(b, tiles)
        c0, r0 = (tile % tiles_x) * TF, (tile // tiles_x) * TF
        for t in range(256):
            dx, dy = t & 15, t >> 4
            c, r = c0 + dx, r0 + dy
            if c < (N + 1) // 2 and r < N // 2:
                for rj, cj in ((r, c), (c, N - 1 - r), (N - 1 - r, N - 1 - c), (N - 1 - c, r)):
                    out.append(g * N * N + rj * N + cj)
        if (N & 1) and tile == 0:
            out.append(g * N * N + (N // 2) * N + N // 2)
    return out


@pytest.mark.parametrize("N", [2, 3, 4, 5, 17, 33, 34, 45, 70, 71, 255])
@pytest.mark.parametrize("split", [1, 3])
def test_fan_turn_kernel_writes_every_pixel_once(N, split):
    """Every pixel of every partial plane (or of the image) is written exactly once
    by the fan-beam quarter-turn kernel's epilogue and centre step."""
    assert sorted(fan_turn_writes(N, split)) == list(range(split * N * N))
