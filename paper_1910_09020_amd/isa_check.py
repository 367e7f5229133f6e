"""Build-time scan of generated gfx950 assembly (host-side tool, never uploaded to GPU runs).

Fails the build if any device code writes through the scalar data cache:
scalar stores, scalar atomics, or scalar-cache write-back/discard.
"""
from __future__ import annotations

import re

FORBIDDEN = re.compile(r"^\s*(s_store_|s_buffer_store|s_scratch_store|s_atomic_|s_buffer_atomic|s_dcache_wb|"
                       r"s_dcache_discard)", re.M)


def scan(path: str) -> list[str]:
    with open(path) as f:
        return sorted(set(FORBIDDEN.findall(f.read())))
