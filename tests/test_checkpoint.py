"""Surrogate checkpoints (host logic): round trip, header and CRC checks."""
import numpy as np
import pytest

from oracle import mlp
from paper_2507_02674_amd.pipeline import pack_checkpoint, unpack_checkpoint


def test_round_trip_is_exact():
    rng = np.random.default_rng(0)
    w = mlp.init(8).astype(np.float32)
    m, v = rng.normal(size=w.size).astype(np.float32), rng.random(w.size).astype(np.float32)
    st = unpack_checkpoint(pack_checkpoint(w, m, v, 123, 8))
    assert st["step"] == 123 and st["K"] == 8
    for a, b in ((st["w"], w), (st["m"], m), (st["v"], v)):
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_corruption_and_bad_headers_are_rejected():
    w = np.arange(16, dtype=np.float32)
    blob = bytearray(pack_checkpoint(w, w, w, 1, 4))
    bad = bytearray(blob)
    bad[40] ^= 0x01
    with pytest.raises(ValueError, match="CRC"):
        unpack_checkpoint(bytes(bad))
    with pytest.raises(ValueError, match="not a surrogate"):
        unpack_checkpoint(b"XXXXXXXX" + bytes(blob[8:]))
    with pytest.raises(ValueError, match="size"):
        unpack_checkpoint(bytes(blob[:-8]))
    ver = bytearray(blob)
    ver[8] = 9  # version field
    with pytest.raises(ValueError, match="version"):
        unpack_checkpoint(bytes(ver))
    with pytest.raises(ValueError):
        pack_checkpoint(w, w[:8], w, 1, 4)
