"""Evaluation keys on disk: a server keeps each client's bootstrapping and
key-switching keys (uint32 [630][6][2][1024] and [1024][8][4][631], the
layouts vlp_keyset_load takes) in an .npz file with a SHA-256 of shapes and
bytes, and refuses a file that does not match it when loading."""
from __future__ import annotations

import hashlib

import numpy as np

BK_SHAPE = (630, 6, 2, 1024)
KSK_SHAPE = (1024, 8, 4, 631)


def _digest(bk: np.ndarray, ksk: np.ndarray) -> str:
    h = hashlib.sha256()
    for a in (bk, ksk):
        h.update(repr(a.shape).encode())
        h.update(np.ascontiguousarray(a, dtype=np.uint32).tobytes())
    return h.hexdigest()


def save_keys(path: str, bk, ksk) -> str:
    """Writes both keys and their digest; returns the digest."""
    bk = np.ascontiguousarray(np.asarray(bk, dtype=np.uint32)).reshape(BK_SHAPE)
    ksk = np.ascontiguousarray(np.asarray(ksk, dtype=np.uint32)).reshape(KSK_SHAPE)
    d = _digest(bk, ksk)
    with open(path, "wb") as f:
        np.savez(f, bk=bk, ksk=ksk, sha256=np.array(d))
    return d


def load_keys(path: str) -> tuple[np.ndarray, np.ndarray]:
    """Reads (bk, ksk); raises ValueError when shapes or digest do not match."""
    with np.load(path, allow_pickle=False) as z:
        bk, ksk, d = z["bk"], z["ksk"], str(z["sha256"])
    if bk.shape != BK_SHAPE or ksk.shape != KSK_SHAPE or bk.dtype != np.uint32 or ksk.dtype != np.uint32:
        raise ValueError("key file %s: unexpected shapes or types" % path)
    if _digest(bk, ksk) != d:
        raise ValueError("key file %s: digest mismatch" % path)
    return bk, ksk
