"""Oracle for the tuning search space — TEST INFRASTRUCTURE ONLY.

The paper's convolution space (Table 1) has block_size_x, block_size_y,
tile_size_x, tile_size_y and three on/off switches (read_only, use_padding,
use_shmem); its restrictions are not printed (Table 3 reports 4,362
configurations for the convolution). The space tuned here is the MI355X
version of that table: block sizes that suit wave64, power-of-two tiles up to
8, LDS halo staging on/off (use_shmem) and filter in constant or global memory
(read_only's analogue), restricted to at most 1024 threads per block.
"""
from __future__ import annotations

import itertools

AXES = (
    ("block_x", (16, 32, 64, 128)),
    ("block_y", (1, 2, 4, 8, 16)),
    ("tile_x", (1, 2, 4, 8)),
    ("tile_y", (1, 2, 4, 8)),
    ("use_lds", (0, 1)),
    ("filter_in_const", (0, 1)),
)

MAX_THREADS = 1024


def product():
    """Every tuple of the unrestricted product, in axis order."""
    return list(itertools.product(*(vals for _, vals in AXES)))


def restricted():
    """Tuples with block_x * block_y <= 1024, in product order."""
    return [c for c in product() if c[0] * c[1] <= MAX_THREADS]


# The hotspot space: the MI355X version of Table 1's hotspot parameters
# (block sizes for wave64, per-thread tiles, temporal tiling factor, step-loop
# unroll, power staging), restricted to 64..1024 threads and a region of
# (block_y*tile_y) x (block_x*tile_x) cells larger than twice the temporal
# factor along both axes (a non-empty output tile once the halo of
# `temporal` cells per side is taken off). Table 1 prints no memory
# restriction; the library also checks a configuration's LDS size against the
# device limit, which no point of these axes reaches, so it is not part of
# this definition.
HOTSPOT_AXES = (
    ("block_x", (16, 32, 64, 128, 256)),
    ("block_y", (1, 2, 4, 8, 16)),
    ("tile_x", (1, 2, 4)),
    ("tile_y", (1, 2, 4)),
    ("temporal", (1, 2, 3, 4, 6, 8)),
    ("unroll_t", (0, 1)),
    ("sh_power", (0, 1)),
)


def hotspot_restricted():
    out = []
    for c in itertools.product(*(vals for _, vals in HOTSPOT_AXES)):
        bx, by, tx, ty, tt = c[:5]
        rows, cols = by * ty, bx * tx
        if not 64 <= bx * by <= MAX_THREADS:
            continue
        if rows <= 2 * tt or cols <= 2 * tt:
            continue
        out.append(c)
    return out
