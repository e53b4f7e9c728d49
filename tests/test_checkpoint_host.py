"""Checkpoint files of ChunkedWave on host tensors (no GPU): the state is
written and read back exactly, into any chunking, and a checkpoint of
another domain, element type or r2 is refused."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def _wave(shape, K, T, dtype="f32", r2=0.25, offset=None):
    from paper_2505_06022_amd.fields import ChunkedWave
    return ChunkedWave(offset or (0,) * len(shape), shape, K, r2, depth=T, device="cpu",
                       dtype=dtype)


@pytest.mark.parametrize("dtype", ["f32", "f64", "bf16"])
def test_save_restore_roundtrip(tmp_path, dtype):
    rng = np.random.default_rng(3)
    shape = (37, 50)
    host = np.float64 if dtype == "f64" else np.float32
    a = rng.standard_normal(shape).astype(host)
    b = rng.standard_normal(shape).astype(host)
    w = _wave(shape, 3, 4, dtype)
    w.scatter(a, b)
    w.n = 41
    path = tmp_path / "state.npz"
    w.save(path)
    w2 = _wave(shape, 2, 8, dtype)  # another chunking and depth
    assert w2.restore(path) == 41 and w2.n == 41
    # the stored values are the fields as held (16-bit: rounded once on scatter)
    assert np.array_equal(w2.gather("prev"), w.gather("prev"))
    assert np.array_equal(w2.gather("cur"), w.gather("cur"))
    if dtype != "bf16":
        assert np.array_equal(w2.gather("cur"), b)


def test_restore_refuses_other_state(tmp_path):
    w = _wave((20, 30), 2, 2)
    w.scatter(np.zeros((20, 30), np.float32), np.ones((20, 30), np.float32))
    path = tmp_path / "s.npz"
    w.save(path)
    with pytest.raises(ValueError):
        _wave((20, 31), 2, 2).restore(path)
    with pytest.raises(ValueError):
        _wave((20, 30), 2, 2, offset=(1, 0)).restore(path)
    with pytest.raises(ValueError):
        _wave((20, 30), 2, 2, dtype="f64").restore(path)
    with pytest.raises(ValueError):
        _wave((20, 30), 2, 2, r2=0.2).restore(path)
