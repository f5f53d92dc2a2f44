"""VDB tree build and coordinate decomposition (oracle, integer-exact).

Follows the [Hash,5,4,3] configuration of Sec. 3.1 (VDB): a sparse root
keyed by level-2 origins, level-2 internal nodes with 32^3 children spanning
4096^3 voxels, level-1 internal nodes with 16^3 children spanning 128^3, and
leaves of 8^3 voxels.  Fig. "vdb" shows the active masks a_l and child masks
c_l that each node carries.

The paper fixes only the fan-outs.  Conventions taken here (the reading
stated for the bit order, which the paper leaves open):
  * leaf origin  = p & ~7,    n0 = (x&7)<<6 | (y&7)<<3 | (z&7)
  * L1 origin    = p & ~127,  n1 = ((x>>3)&15)<<8 | ((y>>3)&15)<<4 | ((z>>3)&15)
  * L2 origin    = p & ~4095, n2 = ((x>>7)&31)<<10 | ((y>>7)&31)<<5 | ((z>>7)&31)
  * root key     = L2 origin; all arithmetic is int32 two's complement, so
    negative coordinates floor towards minus infinity.
  * canonical leaf order: ascending (L2 origin x, y, z, n2, n1), i.e. a
    depth-first walk with children in ascending bit index; voxels inside a
    leaf in ascending n0.
  * mask bit n is bit (n & 63) of 64-bit word (n >> 6).
  * leaf_off is the exclusive prefix sum of per-leaf active counts, with the
    total appended.
"""
import numpy as np

LEAF_LOG2, L1_LOG2, L2_LOG2 = 3, 4, 5          # 8^3, 16^3, 32^3 children
LEAF_DIM, L1_SPAN, L2_SPAN = 8, 128, 4096       # voxel extent of each node kind

SDF, FOG = 0, 1


def active_set_dense(v, origin, kind, band_or_threshold):
    """Active voxels of a dense grid (Sec. 3.2.1, sparse-field training).

    v is a dense array indexed [x][y][z] (x-major, z fastest); origin is the
    index-space coordinate of v[0,0,0].  A narrow-band level set keeps the
    voxels with |phi| <= band (closed interval, reading of the band
    [-3dx, 3dx]); a fog volume keeps the voxels with density > threshold.
    Returns (ijk int32 (N,3), values float64 (N,)) in x-major scan order.
    """
    v = np.asarray(v)
    if kind == SDF:
        act = np.abs(v) <= band_or_threshold
    elif kind == FOG:
        act = v > band_or_threshold
    else:
        raise ValueError("kind must be SDF or FOG")
    idx = np.nonzero(act)
    ijk = np.stack(idx, axis=1).astype(np.int64) + np.asarray(origin, np.int64)[None, :]
    return ijk.astype(np.int32), v[idx].astype(np.float64)


def active_set_sparse(ijk, v, kind, band_or_threshold):
    """The same active rule applied to a sparse voxel list: keeps the rows of
    (ijk, v) that the rule accepts, in the given order.  The comparison is made
    in the precision of v."""
    ijk = np.asarray(ijk, dtype=np.int32).reshape(-1, 3)
    v = np.asarray(v).reshape(-1)
    if kind == SDF:
        act = np.abs(v) <= v.dtype.type(band_or_threshold)
    elif kind == FOG:
        act = v > v.dtype.type(band_or_threshold)
    else:
        raise ValueError("kind must be SDF or FOG")
    return ijk[act], v[act].astype(np.float64)


def decompose(ijk):
    """Per-voxel decomposition into leaf/L1/L2 origins and slot indices."""
    p = np.asarray(ijk, dtype=np.int32)
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    leaf_origin = p & np.int32(~7)
    n0 = ((x & 7) << 6) | ((y & 7) << 3) | (z & 7)
    l1_origin = p & np.int32(~127)
    n1 = (((x >> 3) & 15) << 8) | (((y >> 3) & 15) << 4) | ((z >> 3) & 15)
    l2_origin = p & np.int32(~4095)
    n2 = (((x >> 7) & 31) << 10) | (((y >> 7) & 31) << 5) | ((z >> 7) & 31)
    return dict(leaf_origin=leaf_origin, n0=n0.astype(np.int64), l1_origin=l1_origin,
                n1=n1.astype(np.int64), l2_origin=l2_origin, n2=n2.astype(np.int64))


def n0_to_offset(n0):
    n0 = np.asarray(n0, dtype=np.int64)
    return np.stack([(n0 >> 6) & 7, (n0 >> 3) & 7, n0 & 7], axis=-1)


def n1_to_offset(n1):
    """Voxel offset of leaf slot n1 inside its L1 node."""
    n1 = np.asarray(n1, dtype=np.int64)
    return np.stack([(n1 >> 8) & 15, (n1 >> 4) & 15, n1 & 15], axis=-1) * 8


def _set_bits(words, row, bit):
    """OR bit `bit` into words[row, bit >> 6] (vectorised, duplicates allowed)."""
    np.bitwise_or.at(words, (row, bit >> 6), np.left_shift(np.uint64(1), (bit & 63).astype(np.uint64)))


def build(ijk, values):
    """Build the canonical tree arrays from a sparse active set.

    Duplicate coordinates are rejected.  Returns a dict with
      ijk (N,3) int32, values (N,) float64   -- leaf-major, n0 ascending
      vox_leaf (N,), vox_n0 (N,)             -- owning leaf and slot
      leaf_origin (L,3) int32, leaf_mask (L,8) uint64, leaf_off (L+1,) int64
      leaf_l1 (L,)                           -- parent L1 node index
      l1_origin (L1,3), l1_child (L1,64) uint64, l1_active (L1,64) uint64
      l1_l2 (L1,)                            -- parent L2 node index
      l2_origin (L2,3), l2_child (L2,512) uint64, l2_active (L2,512) uint64
    No tile values exist in a tree built from voxels, so every active mask
    above the leaves is empty.
    """
    ijk = np.asarray(ijk, dtype=np.int32).reshape(-1, 3)
    values = np.asarray(values, dtype=np.float64).reshape(-1)
    assert ijk.shape[0] == values.shape[0]
    d = decompose(ijk)
    l2o, n2, n1, n0 = d["l2_origin"], d["n2"], d["n1"], d["n0"]
    # canonical order: (l2.x, l2.y, l2.z, n2, n1, n0); lexsort takes the last key as primary
    order = np.lexsort((n0, n1, n2, l2o[:, 2], l2o[:, 1], l2o[:, 0]))
    ijk, values = ijk[order], values[order]
    d = {k: v[order] for k, v in d.items()}
    key = np.stack([d["l2_origin"][:, 0].astype(np.int64), d["l2_origin"][:, 1], d["l2_origin"][:, 2],
                    d["n2"], d["n1"], d["n0"]], axis=1)
    if len(key) > 1 and np.any(np.all(key[1:] == key[:-1], axis=1)):
        raise ValueError("duplicate voxel coordinates")
    N = len(values)

    def starts(cols):
        if N == 0:
            return np.zeros(0, dtype=bool)
        s = np.ones(N, dtype=bool)
        s[1:] = np.any(key[1:, :cols] != key[:-1, :cols], axis=1)
        return s

    leaf_start, l1_start, l2_start = starts(5), starts(4), starts(3)
    vox_leaf = np.cumsum(leaf_start) - 1
    vox_l1 = np.cumsum(l1_start) - 1
    vox_l2 = np.cumsum(l2_start) - 1
    L, L1n, L2n = int(leaf_start.sum()), int(l1_start.sum()), int(l2_start.sum())

    leaf_origin = d["leaf_origin"][leaf_start]
    leaf_mask = np.zeros((L, 8), dtype=np.uint64)
    _set_bits(leaf_mask, vox_leaf, d["n0"])
    counts = np.bincount(vox_leaf, minlength=L).astype(np.int64)
    leaf_off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    leaf_l1 = vox_l1[leaf_start]

    l1_origin = d["l1_origin"][l1_start]
    l1_child = np.zeros((L1n, 64), dtype=np.uint64)
    _set_bits(l1_child, leaf_l1, d["n1"][leaf_start])
    l1_l2 = vox_l2[l1_start]

    l2_origin = d["l2_origin"][l2_start]
    l2_child = np.zeros((L2n, 512), dtype=np.uint64)
    _set_bits(l2_child, l1_l2, d["n2"][l1_start])

    return dict(ijk=ijk, values=values, vox_leaf=vox_leaf, vox_n0=d["n0"],
                leaf_origin=leaf_origin, leaf_mask=leaf_mask, leaf_off=leaf_off, leaf_l1=leaf_l1,
                l1_origin=l1_origin, l1_child=l1_child, l1_active=np.zeros_like(l1_child), l1_l2=l1_l2,
                l2_origin=l2_origin, l2_child=l2_child, l2_active=np.zeros_like(l2_child),
                tile_l1=np.zeros(0, np.int64), tile_n1=np.zeros(0, np.int64),
                tile_origin=np.zeros((0, 3), np.int32), tile_value=np.zeros(0, np.float64))


def prune_tiles(tr):
    """Replace every leaf whose 512 voxels are all active and share one value (bit for
    bit) by an active tile of its level-1 node (a constant leaf-sized region that
    carries one value and no leaf node: the active tiles of Sec. 3.3.1, whose values
    the tile value regressor encodes).  The level-1 and upper nodes stay as they are; the
    tile's child bit is cleared and its active-tile bit set.  Tiles keep the
    canonical order of the leaves they replace, i.e. (level-1 node, n1)."""
    L = len(tr["leaf_origin"])
    full = np.all(tr["leaf_mask"] == np.uint64(0xFFFFFFFFFFFFFFFF), axis=1) if L else np.zeros(0, bool)
    const = np.zeros(L, bool)
    for i in np.nonzero(full)[0]:   # one value: identical bit for bit (+0 and -0 differ)
        v = tr["values"][tr["leaf_off"][i]:tr["leaf_off"][i + 1]]
        const[i] = bool(np.all(v == v[0]) and np.all(np.signbit(v) == np.signbit(v[0])))
    tile = full & const
    keep = ~tile
    vox_keep = keep[tr["vox_leaf"]] if len(tr["values"]) else np.zeros(0, bool)
    new_index = np.cumsum(keep) - 1
    leaf_n1 = decompose(tr["leaf_origin"])["n1"] if L else np.zeros(0, np.int64)
    l1_child = tr["l1_child"].copy()
    l1_active = tr["l1_active"].copy()
    for i in np.nonzero(tile)[0]:
        node, n1 = int(tr["leaf_l1"][i]), int(leaf_n1[i])
        l1_child[node, n1 >> 6] &= ~(np.uint64(1) << np.uint64(n1 & 63))
        l1_active[node, n1 >> 6] |= np.uint64(1) << np.uint64(n1 & 63)
    counts = np.diff(tr["leaf_off"])[keep]
    out = dict(tr)
    out.update(ijk=tr["ijk"][vox_keep], values=tr["values"][vox_keep],
               vox_leaf=new_index[tr["vox_leaf"][vox_keep]], vox_n0=tr["vox_n0"][vox_keep],
               leaf_origin=tr["leaf_origin"][keep], leaf_mask=tr["leaf_mask"][keep],
               leaf_off=np.concatenate([[0], np.cumsum(counts)]).astype(np.int64), leaf_l1=tr["leaf_l1"][keep],
               l1_child=l1_child, l1_active=l1_active,
               tile_l1=tr["leaf_l1"][tile].astype(np.int64), tile_n1=leaf_n1[tile].astype(np.int64),
               tile_origin=tr["leaf_origin"][tile],
               tile_value=np.array([tr["values"][tr["leaf_off"][i]] for i in np.nonzero(tile)[0]], np.float64))
    return out


def mask_bits(words, row, n):
    """Bit n of mask row `row` (masks stored as uint64 words), vectorised."""
    row = np.asarray(row, dtype=np.int64)
    n = np.asarray(n, dtype=np.int64)
    return ((words[row, n >> 6] >> (n & 63).astype(np.uint64)) & np.uint64(1)).astype(np.int64)


def popcount64(a):
    a = np.asarray(a, dtype=np.uint64)
    return np.array([bin(int(v)).count("1") for v in a.reshape(-1)], dtype=np.int64).reshape(a.shape)


# --- byte accounting of the explicit tree (Tab. memory_cost) ---------------------------------
# A leaf stores its 512-bit active mask plus a 12-byte origin; its 512 voxel values are
# counted separately (4 bytes each).  An L1 node stores two 4096-bit masks, 4096 4-byte
# child/tile entries and a 12-byte origin; an L2 node two 32768-bit masks, 32768 one-byte
# entries and a 12-byte origin.  These per-node costs reproduce every figure of the table.
LEAF_MASK_BYTES = 512 // 8 + 12                       # 76
L1_NODE_BYTES = 2 * (4096 // 8) + 4096 * 4 + 12       # 17,420
L2_NODE_BYTES = 2 * (32768 // 8) + 32768 * 1 + 12     # 40,972
VOXEL_BYTES = 4
VOXELS_PER_LEAF = 512


def explicit_bytes(n_leaves, n_l1, n_l2):
    """Bytes of a standard [Hash,5,4,3] tree per level (Tab. memory_cost, left block)."""
    return dict(l2=n_l2 * L2_NODE_BYTES, l1=n_l1 * L1_NODE_BYTES,
                leaf_mask=n_leaves * LEAF_MASK_BYTES,
                voxels=n_leaves * VOXELS_PER_LEAF * VOXEL_BYTES)


# A neural level keeps no nodes: its network's parameters (4 bytes each in the
# table's in-memory count, 2 in a 16-bit file) and 12 bytes per patched voxel or
# slot; neural level-1 nodes keep their 12-byte origins (the level-2 masks only
# say which level-1 nodes exist, the origins place them).
PATCH_BYTES = 12
ORIGIN_BYTES = 12


def neural_bytes(n_l2, n_l1, params_l1, patches_l1, params_l0, patches_l0, params_voxels, bytes_per_param=4):
    """Bytes of a [Hash,5,NN(4),NN(3)] NeuralVDB per level (Tab. memory_cost, right block):
    explicit level-2 nodes, then per neural level its parameters and patches."""
    return dict(l2=n_l2 * L2_NODE_BYTES,
                l1=n_l1 * ORIGIN_BYTES + bytes_per_param * params_l1 + PATCH_BYTES * patches_l1,
                leaf_mask=bytes_per_param * params_l0 + PATCH_BYTES * patches_l0,
                voxels=bytes_per_param * params_voxels)
