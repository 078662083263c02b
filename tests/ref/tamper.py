"""Hand-built corrupt archives for the error-path tests.

swap_dependency(a): an archive whose dependency list of one block names a
wrong source block.  One entry d of block b's list is replaced by another
block d2 < b, chosen so that every check reading only the header, directory
and dependency lists still passes (the list stays sorted and distinct, every
entry is earlier than b, b's level is still one more than the highest level
in its list) and so that d is not in the dependency closure of b's new list.
b's matches still read from d, which a range decode of b now never decodes.
"""
from __future__ import annotations

import struct


def _u64(a, o):
    return struct.unpack_from("<Q", a, o)[0]


def swap_dependency(archive: bytes):
    """Returns (tampered archive, b, d, d2)."""
    a = bytearray(archive)
    nb = _u64(a, 32)
    off_dir, off_dep_ptr, off_dep_idx = _u64(a, 64), _u64(a, 72), _u64(a, 80)
    level = [struct.unpack_from("<H", a, off_dir + 32 * b + 20)[0] for b in range(nb)]
    ptr = [_u64(a, off_dep_ptr + 8 * b) for b in range(nb + 1)]
    deps = [[struct.unpack_from("<I", a, off_dep_idx + 4 * k)[0] for k in range(ptr[b], ptr[b + 1])]
            for b in range(nb)]

    def closure(roots):
        seen, stack = set(), list(roots)
        while stack:
            u = stack.pop()
            if u in seen:
                continue
            seen.add(u)
            stack.extend(deps[u])
        return seen

    for b in range(1, nb):
        ds = deps[b]
        for d in ds:
            for d2 in range(b - 1, -1, -1):
                if d2 in ds:
                    continue
                new = sorted([v for v in ds if v != d] + [d2])
                if max(level[v] for v in new) + 1 != level[b]:
                    continue
                if d in closure(new):
                    continue
                for k, v in enumerate(new):
                    struct.pack_into("<I", a, off_dep_idx + 4 * (ptr[b] + k), v)
                return bytes(a), b, d, d2
    raise ValueError("no dependency entry can be swapped consistently")
