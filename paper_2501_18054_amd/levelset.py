"""Level-set optimization on the PNGF state (Supplementary Note 6).

A level-set function phi on the design grid fixes the design (a pixel is at
eps_hi where phi > 0).  Each iteration moves phi along the normal velocity
V = df/dphi = df/deps * deps/dphi, where df/deps comes from the library's
O(N_d) gradient (pngf_gradient, Supplementary Note 5) and deps/dphi is
non-zero only on the boundary band (pixels with a 4-neighbour on the other
side), so few pixels change per iteration.  The pixels whose side of the
boundary changed are flipped together by one block-Woodbury update of C^-1
(pngf_flip_set: the sparse update the note describes), and the iteration is
kept if f improved; otherwise it is undone the same way and the step halves.
phi is re-initialized from the design after every accepted step.

Host logic only: every solve, update and gradient runs in libpngf.  The
design stays binary (no permittivity averaging at the boundary), so each
iteration is an exact PNGF state of a pixel design.
"""
from __future__ import annotations

import numpy as np


def phi_from_bits(bits, side):
    """Initial level set: +1/2 inside eps_hi regions, -1/2 outside."""
    return (np.asarray(bits, dtype=np.float64).reshape(side, side) - 0.5)


def boundary_band(bits, side):
    """Pixels with a 4-neighbour of the other state (the boundary band)."""
    b = np.asarray(bits).reshape(side, side).astype(bool)
    band = np.zeros_like(b)
    band[1:, :] |= b[1:, :] != b[:-1, :]
    band[:-1, :] |= b[:-1, :] != b[1:, :]
    band[:, 1:] |= b[:, 1:] != b[:, :-1]
    band[:, :-1] |= b[:, :-1] != b[:, 1:]
    return band


def run(h, bits0, side, iters=20, step=1.0, min_step=1.0 / 64):
    """Level-set ascent of f from the binary design bits0 on a bound handle
    (FP64_PLAIN or RFORM) of a side x side design region.  Returns a dict
    with the accepted iterations' designs, objectives and changed-pixel
    counts, and the number of rejected trial steps."""
    bits = np.asarray(bits0, dtype=np.uint8).copy()
    h.set_design(bits)
    f = h.evaluate()[0]
    hist = {"f": [f], "bits": [bits.copy()], "changed": [], "rejected": 0}
    for _ in range(iters):
        phi = phi_from_bits(bits, side)
        g = h.gradient().reshape(side, side)           # df/deps
        V = np.where(boundary_band(bits, side), g, 0.0)
        vmax = np.max(np.abs(V))
        if vmax == 0.0:
            break
        accepted = False
        while step >= min_step and not accepted:
            trial = phi + step * V / vmax
            nb = (trial.ravel() > 0).astype(np.uint8)
            changed = np.flatnonzero(nb != bits).astype(np.int32)
            if changed.size == 0:
                break                                   # the step moves nothing
            h.flip_set(changed)
            fn = h.evaluate()[0]
            if fn > f:
                bits, f = nb, fn
                hist["f"].append(f)
                hist["bits"].append(bits.copy())
                hist["changed"].append(int(changed.size))
                accepted = True
            else:
                h.flip_set(changed)                     # undo
                hist["rejected"] += 1
                step *= 0.5
        if not accepted:
            break
    return hist
