"""On-device discrete energy (ccl_wave_energy) against the oracle's
compensated float64 sum of the same definition: random fields in padded
buffers (2D and 3D, every element type), repeated calls bitwise equal, and
the energy of a chunked run's state equal to the oracle's energy of the
oracle's state after the same steps."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

REL = 1e-12  # both sums are float64 over the same float64 terms, in other orders


@pytest.fixture(autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    import paper_2505_06022_amd as ccl
    ccl.lib()  # raises loudly if the library is missing
    yield


def _device_energy(a, b, dtype, r2, pad=5):
    """a, b: host arrays; copied into device buffers whose rows (and planes)
    are padded, the padding filled with NaN (never read)."""
    import paper_2505_06022_amd as ccl
    tdt = {"f32": torch.float32, "f64": torch.float64, "bf16": torch.bfloat16,
           "f16": torch.float16}[dtype]
    full = list(a.shape)
    full[-1] += pad
    if a.ndim == 3:
        full[-2] += 2
    bufs = []
    for h in (a, b):
        t = torch.full(full, float("nan"), dtype=tdt, device="cuda")
        t[tuple(slice(0, n) for n in a.shape)] = torch.from_numpy(h).to(tdt)
        bufs.append(t)
    out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    pitch = [bufs[0].stride(d) for d in range(a.ndim - 1)]
    ccl.ccl_wave_energy(a.shape, pitch, dtype, r2, bufs[0].data_ptr(), bufs[1].data_ptr(),
                        out.data_ptr())
    torch.cuda.synchronize()
    widened = [t[tuple(slice(0, n) for n in a.shape)].double().cpu().numpy() for t in bufs]
    return float(out.item()), widened


@pytest.mark.parametrize("shape", [(37, 50), (1, 1), (300, 1), (9, 11, 13), (2, 1, 600)])
@pytest.mark.parametrize("dtype", ["f32", "f64", "bf16", "f16"])
def test_energy_matches_oracle(shape, dtype):
    print(f"energy case {shape} {dtype}", flush=True)
    rng = np.random.default_rng(len(shape) * 100 + sum(shape))
    a = rng.standard_normal(shape)
    b = a + 0.1 * rng.standard_normal(shape)
    host = np.float64 if dtype == "f64" else np.float32
    e, (wa, wb) = _device_energy(a.astype(host), b.astype(host), dtype, 0.2)
    ref = oracle.energy(wa, wb, 0.2)
    assert np.isfinite(e) and abs(e - ref) <= REL * abs(ref), (e, ref)
    e2, _ = _device_energy(a.astype(host), b.astype(host), dtype, 0.2)
    assert e2 == e  # a fixed summation order


@pytest.mark.parametrize("shape,K,T,r2,steps", [((180, 260), 3, 4, 0.25, 200),
                                               ((24, 40, 50), 2, 6, 0.1, 60)])
def test_chunked_state_energy(shape, K, T, r2, steps):
    from paper_2505_06022_amd.fields import ChunkedWave
    u0 = synth.gaussian_field(shape, 8.0, seed=31)
    cw = ChunkedWave((0,) * len(shape), shape, K, r2, depth=T)
    cw.scatter(u0, u0)
    cw.step(steps)
    e = cw.energy()
    o_prev, o_cur = oracle.wave(u0.copy(), u0, r2, steps)
    ref = oracle.energy(o_cur.astype(np.float64), o_prev.astype(np.float64), r2)
    assert abs(e - ref) <= REL * abs(ref), (e, ref)
    # conserved up to the float32 rounding of the fields
    e0 = oracle.energy(u0.astype(np.float64), u0.astype(np.float64), r2)
    o1p, o1c = oracle.wave(u0.copy(), u0, r2, 1)
    e1 = oracle.energy(o1c.astype(np.float64), o1p.astype(np.float64), r2)
    assert abs(e - e1) <= 1e-4 * abs(e1), (e, e1, e0)
