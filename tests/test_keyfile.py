"""Evaluation keys on disk: round trip, and a changed word or a wrong shape is refused."""
import numpy as np
import pytest

import synth
from paper_2506_12761_amd import keyfile


def test_round_trip_and_tamper_detection(tmp_path):
    bk, ksk = synth.uniform_keys(77)
    path = str(tmp_path / "client.npz")
    d = keyfile.save_keys(path, bk, ksk)
    bk2, ksk2 = keyfile.load_keys(path)
    assert np.array_equal(bk2, bk) and np.array_equal(ksk2, ksk) and len(d) == 64
    # Change one key word but keep the stored digest: refused.
    with np.load(path) as z:
        parts = {k: z[k].copy() for k in z.files}
    parts["ksk"][5, 3, 2, 100] ^= 1
    bad = str(tmp_path / "bad.npz")
    np.savez(bad, **parts)
    with pytest.raises(ValueError, match="digest"):
        keyfile.load_keys(bad)
    parts["ksk"] = parts["ksk"][:512]
    np.savez(bad, **parts)
    with pytest.raises(ValueError, match="shapes"):
        keyfile.load_keys(bad)
