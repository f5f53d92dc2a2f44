"""Sparse domain decomposition with non-learned gates (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

Sec. 3.4 ("Sparse Domain Decomposition", eq. moe): index space is cut into a
regular grid of cubic subdomains of edge S; subdomain D_k is widened on every
side by a halo of h voxels (the paper takes h = 8), so that neighbours overlap.
Subdomains holding no voxel are dropped.  Each remaining subdomain owns its own
network (expert), fed with coordinates normalised to its own bounding box.  A
gate G_k, a clamped tent over the widened box, weights the experts, and the
output is the gate-weighted average of the experts whose gate is non-zero (up
to eight, where eight widened boxes meet).

Readings taken where the paper is silent (every one is listed with the others
in the design notes):
  * grid: cell c (integer triple) has core [o + c S, o + (c+1) S) per axis and
    widened box [o + c S - h, o + (c+1) S + h); o is the grid origin.
  * "empty" means that the core holds no active voxel.  Every active voxel lies
    in the core of exactly one cell, which is therefore kept, so every voxel
    has at least one expert.
  * the tent is evaluated at the voxel centre p + 1/2.  With t the distance of
    the centre from the lower face of the widened box, per axis
    g(t) = min(t, S + 2h - t, 2h) / (2h): it rises across the 2h-wide band where
    two widened boxes overlap and is 1 in between.  In that band the two
    neighbours' tents sum to 1.  The 3-D gate is the product over the axes.
  * the paper states eq. moe as a plain sum and, in words, a weighted average.
    The average sum_k G_k E_k / sum_k G_k is taken.  It equals eq. moe wherever
    the gates sum to 1, and it stays a convex blend next to dropped cells and
    at the outer faces of the grid.
  * expert input: x = (p - lo_k + 1/2) / D_k, with lo_k the lower corner of the
    widened box and D_k = S + 2h its edge ("normalized coordinates between
    [0, 1] for the given subdomain bounding box").
  * S >= 2h (so a voxel meets at most two cells per axis) and h >= 1.
"""
import numpy as np

from . import mlp


def check_geometry(S, h):
    if not (int(h) >= 1 and int(S) >= 2 * int(h)):
        raise ValueError("subdomains need halo >= 1 and size >= 2 * halo")


def core_cell(ijk, origin, S):
    """Cell whose core holds each voxel: floor((p - o) / S) per axis."""
    p = np.asarray(ijk, np.int64).reshape(-1, 3)
    return np.floor_divide(p - np.asarray(origin, np.int64), int(S))


def kept_cells(ijk, origin, S):
    """Cells whose core holds at least one voxel, ascending in (cx, cy, cz)."""
    c = core_cell(ijk, origin, S)
    if len(c) == 0:
        return np.zeros((0, 3), np.int64)
    return np.unique(c, axis=0)


def widened_box(cell, origin, S, h):
    """Lower corner and edge of a cell's widened box (core plus halo)."""
    lo = np.asarray(origin, np.int64) + np.asarray(cell, np.int64) * int(S) - int(h)
    return lo, int(S) + 2 * int(h)


def in_widened_box(ijk, cell, origin, S, h):
    p = np.asarray(ijk, np.int64).reshape(-1, 3)
    lo, D = widened_box(cell, origin, S, h)
    return np.all((p >= lo) & (p < lo + D), axis=1)


def gate(ijk, cell, origin, S, h):
    """Clamped tent G_k at the voxel centres (zero outside the widened box)."""
    p = np.asarray(ijk, np.int64).reshape(-1, 3)
    lo, D = widened_box(cell, origin, S, h)
    t = p.astype(np.float64) + 0.5 - lo.astype(np.float64)
    g = np.minimum(np.minimum(t, D - t), 2.0 * h) / (2.0 * h)
    g = np.clip(g, 0.0, None)
    return np.prod(g, axis=1) * in_widened_box(p, cell, origin, S, h)


def gate_leaf_slot(o, cell, origin, S, h):
    """Clamped tent G_k at the centres o + 4 of the leaf slots at origins o (zero
    where the slot's 8^3 block is not wholly inside the widened box)."""
    o = np.asarray(o, np.int64).reshape(-1, 3)
    lo, D = widened_box(cell, origin, S, h)
    t = o.astype(np.float64) + 4.0 - lo.astype(np.float64)
    g = np.minimum(np.minimum(t, D - t), 2.0 * h) / (2.0 * h)
    g = np.clip(g, 0.0, None)
    inside = np.all((o >= lo) & (o + 8 <= lo + D), axis=1)
    return np.prod(g, axis=1) * inside


def decode_moe_l1(slot_origins, experts, origin, S, h):
    """Blended level-1 classes at leaf slots (origins o): the experts' three logits
    at x = (o - lo + 4) / D averaged with the gates at the slot centres, then the
    argmax (ties to the lowest class).  Returns (classes, blended logits)."""
    check_geometry(S, h)
    o = np.asarray(slot_origins, np.int64).reshape(-1, 3)
    num = np.zeros((len(o), 3))
    den = np.zeros(len(o))
    for e in experts:
        g = gate_leaf_slot(o, e["cell"], origin, S, h)
        sel = g > 0
        if not sel.any():
            continue
        x = mlp.normalize_leaf_slot(o[sel], e["lo"], e["D"])
        y = mlp.predict(mlp.unflatten(e["theta"], e["shapes"]), x, e["B"])
        num[sel] += g[sel][:, None] * y
        den[sel] += g[sel]
    logits = np.full((len(o), 3), np.nan)
    ok = den > 0
    logits[ok] = num[ok] / den[ok][:, None]
    return np.argmax(np.where(np.isnan(logits), -np.inf, logits), axis=1), logits


def decode_moe_tiles(tile_origins, experts, origin, S, h):
    """Blended values of active tiles (Sec. 3.3.1 tile values under the
    decomposition of Sec. 3.4): each expert's tile value regressor at the tile's
    leaf-slot centre, x = (o - lo + 4) / D, scaled by the expert's value scale and
    averaged with the gates at the slot centres (those of decode_moe_l1).  Tiles
    that no gate covers get NaN."""
    check_geometry(S, h)
    o = np.asarray(tile_origins, np.int64).reshape(-1, 3)
    num = np.zeros(len(o))
    den = np.zeros(len(o))
    for e in experts:
        g = gate_leaf_slot(o, e["cell"], origin, S, h)
        sel = g > 0
        if not sel.any():
            continue
        x = mlp.normalize_leaf_slot(o[sel], e["lo"], e["D"])
        y = mlp.predict(mlp.unflatten(e["theta"], e["shapes"]), x, e["B"])[:, 0]
        num[sel] += g[sel] * y * float(e["scale"])
        den[sel] += g[sel]
    out = np.full(len(o), np.nan)
    ok = den > 0
    out[ok] = num[ok] / den[ok]
    return out


def subdomain_voxels(ijk, values, cell, origin, S, h):
    """Voxels (coordinates, values) of the widened box of `cell`: the training
    set of its expert."""
    m = in_widened_box(ijk, cell, origin, S, h)
    return np.asarray(ijk)[m], np.asarray(values)[m]


def decode_moe(ijk, experts, origin, S, h):
    """Blended decode (eq. moe, as a weighted average) at voxels ijk.

    experts: list of dicts with keys cell, theta, shapes, B, lo, D, scale (the
    expert's flat parameters, layer shapes, Fourier matrix, normalisation box
    and value scale).  Every expert is tried against every voxel: the gate
    alone decides who contributes.  Voxels that no gate covers get NaN."""
    check_geometry(S, h)
    p = np.asarray(ijk, np.int64).reshape(-1, 3)
    num = np.zeros(len(p))
    den = np.zeros(len(p))
    for e in experts:
        g = gate(p, e["cell"], origin, S, h)
        sel = g > 0
        if not sel.any():
            continue
        x = mlp.normalize_voxel(p[sel], e["lo"], e["D"])
        y = mlp.predict(mlp.unflatten(e["theta"], e["shapes"]), x, e["B"])[:, 0]
        num[sel] += g[sel] * y * float(e["scale"])
        den[sel] += g[sel]
    out = np.full(len(p), np.nan)
    ok = den > 0
    out[ok] = num[ok] / den[ok]
    return out
