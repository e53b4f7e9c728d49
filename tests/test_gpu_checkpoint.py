"""Checkpoint / resume on the GPU: 2k leapfrog steps in one go equal k
steps, a checkpoint, a fresh set of chunk buffers (another chunking and
depth where the result does not depend on them) restored from it and k
more steps, bitwise, and both equal the oracle."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    import paper_2505_06022_amd as ccl
    ccl.lib()  # raises loudly if the library is missing
    yield


CASES = [
    # shape, r2, k, (K, T) before the checkpoint, (K, T) after, dtype
    ((150, 260), 0.25, 23, (3, 5), (2, 8), "f32"),
    ((20, 40, 70), 0.1, 13, (2, 6), (3, 4), "f32"),
    ((90, 130), 0.25, 17, (2, 3), (4, 7), "f64"),
    ((90, 130), 0.25, 12, (3, 4), (2, 4), "bf16"),  # k on a block boundary, same T
]


@pytest.mark.parametrize("shape,r2,k,before,after,dtype", CASES)
def test_resume_equals_uninterrupted(tmp_path, shape, r2, k, before, after, dtype):
    from paper_2505_06022_amd.fields import ChunkedWave
    print(f"checkpoint case {shape} {dtype} k={k} {before} -> {after}", flush=True)
    u0 = synth.gaussian_field(shape, 7.0, seed=21)
    host = u0.astype(np.float64) if dtype == "f64" else u0
    zero = (0,) * len(shape)

    whole = ChunkedWave(zero, shape, before[0], r2, depth=before[1], dtype=dtype)
    whole.scatter(host, host)
    whole.step(2 * k)
    ref_prev, ref_cur = whole.gather("prev"), whole.gather("cur")
    del whole

    first = ChunkedWave(zero, shape, before[0], r2, depth=before[1], dtype=dtype)
    first.scatter(host, host)
    first.step(k)
    path = tmp_path / "state.npz"
    first.save(path)
    del first
    second = ChunkedWave(zero, shape, after[0], r2, depth=after[1], dtype=dtype, fill=float("nan"))
    assert second.restore(path) == k
    second.step(k)
    assert second.n == 2 * k
    got_prev, got_cur = second.gather("prev"), second.gather("cur")
    assert np.array_equal(got_cur, ref_cur) and np.array_equal(got_prev, ref_prev)

    if dtype == "bf16":
        o_prev, o_cur = oracle.wave_stored(host.copy(), host, r2, 2 * k, before[1], dtype)
    else:
        o_prev, o_cur = oracle.wave(host.copy(), host, r2, 2 * k)
    assert np.array_equal(got_cur, o_cur) and np.array_equal(got_prev, o_prev)
