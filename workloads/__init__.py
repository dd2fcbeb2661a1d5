"""Seeded synthetic inputs for the 2D TM (Ez) pixel inverse-design problems.

This module only draws and lays out input arrays (permittivity maps, design
masks, source and output profiles, frequencies, initial designs, sweep
orders).  It contains none of the method's arithmetic: no operator, no solve,
no Green function, no objective.  Both the CPU oracle and the GPU library
consume exactly these arrays.

Conventions (shared by every consumer):
  * 2D arrays are shaped (ny, nx) and indexed [j, i]; i is x, j is y.
    The flat node index is n = j*nx + i (row-major, y outer, x inner).
  * Points are written (x, y) = (i, j).
  * Lengths are in units of the free-space wavelength lambda0 at f0, so
    k0(f) = 2*pi*f/f0 and the grid step h is a fraction of lambda0.
  * Design pixels are enumerated in the same row-major order restricted to
    the design mask; pixel m <-> m-th nonzero of design_mask.ravel().
  * Design bit p_m = 1 means eps_hi, 0 means eps_lo; eps_static holds eps_lo
    on design cells.  For problems with pixel_kind == PEC, bit 1 means a
    perfectly conducting pixel (Ez = 0 on that node) and eps_hi is unused.
  * All randomness comes from numpy Generator(PCG64(...)) keyed on the seed.

The five standard workloads follow the stated test configurations:
  0: 48x48 grid, 10x10 design, point source -> point |Ez|^2, one sweep.
  1: 256x256 grid, 40x40 design (eps 11.7), Gaussian line source -> Gaussian
     overlap, five sweeps.
  2: 48 problems of uneven size and 1-4 frequencies (batching).
  3: config-1-type problems with training / held-out seeds (learned proposer).
  4: 640x640 grid, 80x80 design, eight frequencies, normalized transmission.
plus ``metal`` / ``tiny_metal``: the same kind of problem with perfectly
conducting (PEC) pixels, the paper's own device type; and ``tiles1`` /
``with_tiles``: searches whose flips are groups of M pixels (tiles of several
nodes, optionally tied by mirror symmetry).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

POINT_INTENSITY = 0
OVERLAP_INTENSITY = 1
MEAN_TRANSMISSION = 2

DIELECTRIC = 0
PEC = 1


@dataclass
class Problem:
    """Plain arrays describing one inverse-design problem (no derived data)."""

    name: str
    seed: int
    nx: int
    ny: int
    npml: int
    h: float                    # grid step in units of lambda0
    eps_static: np.ndarray      # (ny, nx) float64; design cells hold eps_lo
    design_mask: np.ndarray     # (ny, nx) uint8
    eps_lo: float
    eps_hi: float
    k0: np.ndarray              # (nfreq,) float64, k0 = 2*pi*f/f0
    src: np.ndarray             # (nfreq, ny*nx) complex128 current density J
    w: np.ndarray               # (nobj, ny*nx) complex128 output functional
    objective_kind: int
    obj_norm: np.ndarray        # (nfreq,) float64 normalizers (1.0 unless set)
    init_bits: np.ndarray       # (n_d,) uint8 initial design
    perms: np.ndarray           # (n_sweeps, n_d) int32 sweep visiting orders
    design_origin: tuple = (0, 0)   # (i0, j0) of the square design region
    design_side: int = 0
    log: list = field(default_factory=list)
    pixel_kind: int = DIELECTRIC    # DIELECTRIC (eps_lo/eps_hi) or PEC pixels
    tiles: np.ndarray = None        # optional (n_tiles, M) pixel groups, -1 padded
    tile_perms: np.ndarray = None   # (n_sweeps, n_tiles) visiting orders of the tiles

    @property
    def nfreq(self) -> int:
        return int(self.k0.shape[0])

    @property
    def n_d(self) -> int:
        return int(self.design_mask.sum())

    @property
    def n_sweeps(self) -> int:
        return int(self.perms.shape[0])

    def design_indices(self) -> np.ndarray:
        """Flat node indices (n = j*nx + i) of design pixels in pixel order."""
        return np.flatnonzero(self.design_mask.ravel()).astype(np.int64)


def _rng(*key) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(list(key)))


def _gaussian(n: int, sigma: float) -> np.ndarray:
    """Gaussian amplitude profile over n cells, centered at (n-1)/2."""
    y = np.arange(n, dtype=np.float64)
    yc = (n - 1) / 2.0
    return np.exp(-((y - yc) ** 2) / (2.0 * sigma * sigma))


def _rect_clear(x0, y0, x1, y1, keepouts, margin):
    """True if [x0,x1)x[y0,y1) keeps `margin` cells from every keep-out rect."""
    for (a0, b0, a1, b1) in keepouts:
        if x0 < a1 + margin and a0 - margin < x1 and y0 < b1 + margin and b0 - margin < y1:
            return False
    return True


def _place_rects(rng, nx, ny, npml, keepouts, count, size_fn, eps_map, eps_val,
                 margin, log, tries=1000):
    placed = []
    for r in range(count):
        ok = False
        for _ in range(tries):
            w, hgt = size_fn(rng)
            lo_x, hi_x = npml, nx - npml - w
            lo_y, hi_y = npml, ny - npml - hgt
            if hi_x < lo_x or hi_y < lo_y:
                break
            x0 = int(rng.integers(lo_x, hi_x + 1))
            y0 = int(rng.integers(lo_y, hi_y + 1))
            if _rect_clear(x0, y0, x0 + w, y0 + hgt, keepouts, margin):
                eps_map[y0:y0 + hgt, x0:x0 + w] = eps_val
                placed.append((x0, y0, x0 + w, y0 + hgt))
                ok = True
                break
        if not ok:
            log.append(f"feature {r} skipped: no placement after {tries} tries")
    return placed


def _sweep_perms(seed: int, n_sweeps: int, n_d: int) -> np.ndarray:
    out = np.empty((n_sweeps, n_d), dtype=np.int32)
    for s in range(n_sweeps):
        out[s] = _rng(seed, 7000 + s).permutation(n_d).astype(np.int32)
    return out


def _square_problem(name, seed, n, npml, h, side, eps_hi, k0s, src_pts, out_pts,
                    src_profile, out_profile, objective_kind, n_sweeps,
                    feature, rng, i0=None, j0=None, ny=None):
    """Common builder: square grid, centered square design, line/point ports."""
    nx = n
    ny = n if ny is None else ny
    if i0 is None:
        i0 = (nx - side) // 2
    if j0 is None:
        j0 = (ny - side) // 2
    eps = np.ones((ny, nx), dtype=np.float64)
    mask = np.zeros((ny, nx), dtype=np.uint8)
    mask[j0:j0 + side, i0:i0 + side] = 1
    log = []
    keepouts = [(i0, j0, i0 + side, j0 + side)]
    for (x, ya, yb) in list(src_pts) + list(out_pts):
        keepouts.append((x, ya, x + 1, yb))
    feature(rng, nx, ny, npml, keepouts, eps, log)
    nf = len(k0s)
    src = np.zeros((nf, ny * nx), dtype=np.complex128)
    for (x, ya, yb) in src_pts:
        prof = src_profile(yb - ya)
        for fi in range(nf):
            for t, y in enumerate(range(ya, yb)):
                src[fi, y * nx + x] = prof[t]
    w = np.zeros((1, ny * nx), dtype=np.complex128)
    for (x, ya, yb) in out_pts:
        prof = out_profile(yb - ya)
        for t, y in enumerate(range(ya, yb)):
            w[0, y * nx + x] = prof[t]
    n_d = side * side
    init_bits = (rng.random(n_d) < 0.5).astype(np.uint8)
    perms = _sweep_perms(seed, n_sweeps, n_d)
    return Problem(name=name, seed=seed, nx=nx, ny=ny, npml=npml, h=h,
                   eps_static=eps, design_mask=mask, eps_lo=1.0, eps_hi=eps_hi,
                   k0=np.asarray(k0s, dtype=np.float64), src=src, w=w,
                   objective_kind=objective_kind,
                   obj_norm=np.ones(nf, dtype=np.float64), init_bits=init_bits,
                   perms=perms, design_origin=(i0, j0), design_side=side, log=log)


def _block_feature(eps_val=2.2, count=1, margin=2):
    def f(rng, nx, ny, npml, keepouts, eps, log):
        _place_rects(rng, nx, ny, npml, keepouts, count,
                     lambda r: (int(r.integers(3, 9)), int(r.integers(3, 9))),
                     eps, eps_val, margin, log)
    return f


def _slab_feature(scale=1.0, eps_val=2.2, margin=2):
    def size(r):
        thick = int(round(int(r.integers(2, 7)) * scale))
        length = int(round(int(r.integers(20, 81)) * scale))
        if r.random() < 0.5:
            return (length, thick)
        return (thick, length)

    def f(rng, nx, ny, npml, keepouts, eps, log):
        count = int(rng.integers(3, 7))
        _place_rects(rng, nx, ny, npml, keepouts, count, size, eps, eps_val,
                     margin, log)
    return f


def config0(seed: int = 0) -> Problem:
    """48x48, 8-cell PML, 10x10 design at [19,29)^2, eps in {1,4}."""
    rng = _rng(seed, 0)
    one = lambda n: np.ones(n)
    return _square_problem(
        "config0", seed, 48, 8, 1.0 / 20.0, 10, 4.0, [2.0 * math.pi],
        src_pts=[(10, 24, 25)], out_pts=[(38, 24, 25)],
        src_profile=one, out_profile=one, objective_kind=POINT_INTENSITY,
        n_sweeps=1, feature=_block_feature(), rng=rng)


def config1(seed: int = 1, n_sweeps: int = 5) -> Problem:
    """256x256, 12-cell PML, 40x40 design at [108,148)^2, eps in {1,11.7}."""
    rng = _rng(seed, 1)
    side = 40
    i0 = (256 - side) // 2
    j0 = i0
    g = lambda n: _gaussian(n, 6.0)
    return _square_problem(
        "config1", seed, 256, 12, 1.0 / 20.0, side, 11.7, [2.0 * math.pi],
        src_pts=[(84, j0, j0 + side)], out_pts=[(172, j0, j0 + side)],
        src_profile=g, out_profile=g, objective_kind=OVERLAP_INTENSITY,
        n_sweeps=n_sweeps, feature=_slab_feature(), rng=rng)


def config2_problem(seed: int, n_sweeps: int = 20) -> Problem:
    """One problem of the batching workload (seeds 1000..1047)."""
    rng = _rng(seed, 2)
    n = int(rng.integers(96, 321))
    side = int(rng.integers(16, 57))
    eps_hi = 4.0 if rng.random() < 0.5 else 11.7
    nf = int(rng.integers(1, 5))
    k0s = [2.0 * math.pi * float(rng.uniform(0.9, 1.1)) for _ in range(nf)]
    i0 = (n - side) // 2
    one = lambda m: np.ones(m)
    return _square_problem(
        f"config2_s{seed}", seed, n, 10, 1.0 / 20.0, side, eps_hi, k0s,
        src_pts=[(i0 - 6, n // 2, n // 2 + 1)],
        out_pts=[(i0 + side + 5, n // 2, n // 2 + 1)],
        src_profile=one, out_profile=one, objective_kind=POINT_INTENSITY,
        n_sweeps=n_sweeps, feature=_block_feature(), rng=rng)


def config2(seeds=range(1000, 1048), n_sweeps: int = 20):
    return [config2_problem(s, n_sweeps) for s in seeds]


CONFIG3_TRAIN_SEEDS = tuple(range(2000, 2064))
CONFIG3_EVAL_SEEDS = tuple(range(3000, 3008))


def config3_problem(seed: int, n_sweeps: int = 5) -> Problem:
    p = config1(seed, n_sweeps)
    p.name = f"config3_s{seed}"
    return p


def config4(seed: int = 4, n_sweeps: int = 20) -> Problem:
    """640x640, 16-cell PML, h = lambda0/25, 80x80 design, 8 frequencies."""
    rng = _rng(seed, 4)
    side = 80
    i0 = (640 - side) // 2
    j0 = i0
    k0s = [2.0 * math.pi * (0.9 + 0.2 * i / 7.0) for i in range(8)]
    g = lambda n: _gaussian(n, 12.0)
    return _square_problem(
        "config4", seed, 640, 16, 1.0 / 25.0, side, 11.7, k0s,
        src_pts=[(i0 - 40, j0, j0 + side)], out_pts=[(i0 + side + 40, j0, j0 + side)],
        src_profile=g, out_profile=g, objective_kind=MEAN_TRANSMISSION,
        n_sweeps=n_sweeps, feature=_slab_feature(scale=640.0 / 256.0), rng=rng)


def config4_scaled(seed: int = 4, n: int = 160, side: int = 24, n_sweeps: int = 2) -> Problem:
    """Workload 4's broadband setting at a size the oracle can search: h =
    lambda0/25, 16-cell PML, eight frequencies over 0.9-1.1 f0, Gaussian line
    source and overlap output scaled with the design, mean over frequencies,
    slab background scaled like workload 4; a 160x160 grid with a 24x24
    design instead of 640x640 with 80x80."""
    rng = _rng(seed, 44)
    i0 = (n - side) // 2
    j0 = i0
    k0s = [2.0 * math.pi * (0.9 + 0.2 * i / 7.0) for i in range(8)]
    g = lambda m: _gaussian(m, 12.0 * side / 80.0)
    return _square_problem(
        "config4_scaled", seed, n, 16, 1.0 / 25.0, side, 11.7, k0s,
        src_pts=[(i0 - 20, j0, j0 + side)], out_pts=[(i0 + side + 20, j0, j0 + side)],
        src_profile=g, out_profile=g, objective_kind=MEAN_TRANSMISSION,
        n_sweeps=n_sweeps, feature=_slab_feature(scale=n / 256.0), rng=rng)


def tiny(seed: int = 0, n: int = 20, npml: int = 4, side: int = 3,
         eps_hi: float = 4.0, nfreq: int = 1, n_sweeps: int = 3,
         static_block: bool = True) -> Problem:
    """Small problem for brute-force checks (full enumeration is cheap)."""
    rng = _rng(seed, 99)
    i0 = (n - side) // 2
    k0s = [2.0 * math.pi * (1.0 + 0.05 * f) for f in range(nfreq)]
    one = lambda m: np.ones(m)
    feat = _block_feature() if static_block else (lambda *a: None)
    sx = max(npml + 1, i0 - 3)
    ox = min(n - npml - 2, i0 + side + 2)
    return _square_problem(
        f"tiny_s{seed}", seed, n, npml, 1.0 / 20.0, side, eps_hi, k0s,
        src_pts=[(sx, n // 2, n // 2 + 1)], out_pts=[(ox, n // 2, n // 2 + 1)],
        src_profile=one, out_profile=one, objective_kind=POINT_INTENSITY,
        n_sweeps=n_sweeps, feature=feat, rng=rng)


def metal(seed: int = 5, n: int = 96, side: int = 24, nfreq: int = 1,
          n_sweeps: int = 3, fill: float = 0.3) -> Problem:
    """Pixelated metal device: 96x96 grid, 10-cell PML, 24x24 design of PEC
    pixels on eps_lo = 1, one dielectric block outside the design, point
    source -> point |Ez|^2; about 30% of the pixels start as metal."""
    rng = _rng(seed, 5)
    i0 = (n - side) // 2
    k0s = [2.0 * math.pi * (1.0 + 0.04 * f) for f in range(nfreq)]
    one = lambda m: np.ones(m)
    p = _square_problem(
        f"metal_s{seed}", seed, n, 10, 1.0 / 20.0, side, 1.0, k0s,
        src_pts=[(i0 - 8, n // 2, n // 2 + 1)], out_pts=[(i0 + side + 8, n // 2, n // 2 + 1)],
        src_profile=one, out_profile=one, objective_kind=POINT_INTENSITY,
        n_sweeps=n_sweeps, feature=_block_feature(), rng=rng)
    p.init_bits = (_rng(seed, 55).random(p.n_d) < fill).astype(np.uint8)
    p.pixel_kind = PEC
    return p


def tiny_metal(seed: int = 0, n: int = 20, npml: int = 4, side: int = 3,
               nfreq: int = 1, n_sweeps: int = 3) -> Problem:
    """tiny() with PEC pixels."""
    p = tiny(seed=seed, n=n, npml=npml, side=side, eps_hi=1.0, nfreq=nfreq,
             n_sweeps=n_sweeps)
    p.name = f"tiny_metal_s{seed}"
    p.pixel_kind = PEC
    return p


def tile_groups(side: int, a: int, mirror: bool = False) -> np.ndarray:
    """Pixel groups flipped together, for a side x side design region: a x a
    blocks of pixels (ragged at the far edges when a does not divide side);
    with ``mirror`` each block is tied to its mirror image about the region's
    vertical axis (a design kept symmetric in x).  Returns (n_groups, M) int32
    pixel ids, -1 padded, in row-major block order."""
    nb = (side + a - 1) // a
    blocks = {}
    for bj in range(nb):
        for bi in range(nb):
            pix = [j * side + i for j in range(bj * a, min(side, bj * a + a))
                   for i in range(bi * a, min(side, bi * a + a))]
            blocks[(bi, bj)] = pix
    groups = []
    for bj in range(nb):
        for bi in range(nb):
            if mirror:
                mi = nb - 1 - bi
                if mi < bi:
                    continue
                pix = blocks[(bi, bj)] + (blocks[(mi, bj)] if mi != bi else [])
            else:
                pix = blocks[(bi, bj)]
            groups.append(pix)
    M = max(len(g) for g in groups)
    out = np.full((len(groups), M), -1, dtype=np.int32)
    for t, g in enumerate(groups):
        out[t, :len(g)] = g
    return out


def with_tiles(p: Problem, a: int, mirror: bool = False, n_sweeps=None) -> Problem:
    """Attach tile groups (tile_groups) and per-sweep visiting orders of the
    groups to a square-design problem."""
    side = p.design_side
    p.tiles = tile_groups(side, a, mirror)
    ns = p.n_sweeps if n_sweeps is None else n_sweeps
    nt = p.tiles.shape[0]
    p.tile_perms = np.stack([_rng(p.seed, 8000 + s).permutation(nt).astype(np.int32)
                             for s in range(ns)]) if ns > 0 else np.zeros((0, nt), np.int32)
    p.name = f"{p.name}_tiles{a}{'m' if mirror else ''}"
    return p


def tiles1(seed: int = 1) -> Problem:
    """Workload 1 (40x40 design) searched over 4x4-pixel tiles (M = 16, 100
    tiles), five sweeps."""
    return with_tiles(config1(seed, n_sweeps=5), 4)


def make_config(i: int, seed=None):
    """Return the standard workload i (a Problem, or a list for config 2)."""
    if i == 0:
        return config0(0 if seed is None else seed)
    if i == 1:
        return config1(1 if seed is None else seed)
    if i == 2:
        return config2()
    if i == 3:
        return config3_problem(CONFIG3_EVAL_SEEDS[0] if seed is None else seed)
    if i == 4:
        return config4(4 if seed is None else seed)
    raise ValueError(f"unknown config {i}")
