"""Tile binning written as its plain definition (Sec. 3.1: each 2D Gaussian
is "projected onto different image tiles" and then "sorted").

  tile_mask_counts  number of masked pixels per tile; a tile is active when
                    the count is non-zero (only masked pixels are rendered,
                    Sec. 1 and Sec. 5.3)
  emit_and_sort     for every record in index order and every active tile of
                    its tile rectangle in row-major order, one pair
                    key = (global tile id << 32) | depth-key bits,
                    value = record id; then a stable sort by key and the
                    per-tile [start, end) ranges (empty tiles [0, 0)).

All integer work; the GPU must match it bit for bit.  The sort is numpy's
stable argsort (a library routine).
"""
import numpy as np


def tile_grid(width, height, tile):
    return (width + tile - 1) // tile, (height + tile - 1) // tile


def tile_mask_counts(mask, width, height, tile):
    """uint32 [tiles_y * tiles_x] masked-pixel count per tile (row-major)."""
    tx, ty = tile_grid(width, height, tile)
    m = np.ones((height, width), np.int64) if mask is None else np.asarray(mask).astype(np.int64)
    pad = np.zeros((ty * tile, tx * tile), np.int64)
    pad[:height, :width] = m != 0
    c = pad.reshape(ty, tile, tx, tile).sum(axis=(1, 3))
    return c.reshape(-1).astype(np.uint32)


def emit_and_sort(rects, depth_bits, valid, record_render, render_tiles, render_tile_offset,
                  active):
    """Reference binning.

    rects          int [n, 4] per record (x0, y0, x1, y1), half-open tile rect
    depth_bits     uint32 [n] depth-key bits
    valid          bool [n] record takes part
    record_render  int [n] render index of each record
    render_tiles   list of (tiles_x, tiles_y) per render
    render_tile_offset  int [n_renders] first global tile id of each render
    active         bool [total_tiles] active flag per global tile
    Returns (keys uint64 [K], values uint32 [K], ranges uint32 [total_tiles, 2]).
    """
    keys, vals = [], []
    n = len(depth_bits)
    for i in range(n):
        if not valid[i]:
            continue
        r = int(record_render[i])
        tx_n, _ = render_tiles[r]
        x0, y0, x1, y1 = (int(v) for v in rects[i])
        for ty in range(y0, y1):
            for tx in range(x0, x1):
                gt = int(render_tile_offset[r]) + ty * tx_n + tx
                if active[gt]:
                    keys.append((gt << 32) | int(depth_bits[i]))
                    vals.append(i)
    keys = np.asarray(keys, dtype=np.uint64)
    vals = np.asarray(vals, dtype=np.uint32)
    order = np.argsort(keys, kind="stable")
    keys, vals = keys[order], vals[order]
    total = len(active)
    ranges = np.zeros((total, 2), np.uint32)
    tiles = (keys >> np.uint64(32)).astype(np.int64)
    for k in range(len(keys)):
        t = tiles[k]
        if k == 0 or tiles[k - 1] != t:
            ranges[t, 0] = k
        if k == len(keys) - 1 or tiles[k + 1] != t:
            ranges[t, 1] = k + 1
    return keys, vals, ranges


def emit_and_sort_fast(rects, depth_bits, valid, record_render, render_tiles,
                       render_tile_offset, active):
    """Same result as ``emit_and_sort`` with the per-record loops expanded by
    numpy (for inputs with millions of pairs)."""
    idx = np.flatnonzero(valid)
    r = np.asarray(record_render)[idx]
    rc = np.asarray(rects, dtype=np.int64)[idx]
    wx = np.maximum(rc[:, 2] - rc[:, 0], 0)
    wy = np.maximum(rc[:, 3] - rc[:, 1], 0)
    cnt = wx * wy
    owner = np.repeat(np.arange(len(idx)), cnt)
    local = np.arange(int(cnt.sum())) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    txs = np.asarray([t[0] for t in render_tiles], dtype=np.int64)
    tx = rc[owner, 0] + local % wx[owner]
    ty = rc[owner, 1] + local // wx[owner]
    gt = np.asarray(render_tile_offset, dtype=np.int64)[r[owner]] + ty * txs[r[owner]] + tx
    keep = np.asarray(active)[gt]
    gt, owner = gt[keep], owner[keep]
    keys = (gt.astype(np.uint64) << np.uint64(32)) | np.asarray(depth_bits, np.uint64)[idx[owner]]
    vals = idx[owner].astype(np.uint32)
    order = np.argsort(keys, kind="stable")
    keys, vals = keys[order], vals[order]
    total = len(active)
    tiles = (keys >> np.uint64(32)).astype(np.int64)
    ranges = np.zeros((total, 2), np.uint32)
    if len(keys):
        first = np.ones(len(keys), bool)
        first[1:] = tiles[1:] != tiles[:-1]
        last = np.ones(len(keys), bool)
        last[:-1] = tiles[1:] != tiles[:-1]
        ranges[tiles[first], 0] = np.flatnonzero(first)
        ranges[tiles[last], 1] = np.flatnonzero(last) + 1
    return keys, vals, ranges
