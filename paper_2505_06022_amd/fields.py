"""Chunk buffers in device memory for the binding (PyTorch as allocator).

``ChunkedWave`` splits a domain with ccl_split_range, sizes every chunk's
buffers with ccl_region_of (NEIGHBORHOOD(T) against the virtual buffer),
allocates them with torch, scatters an initial state into the chunk cells
and gathers the chunk cells back.  Stepping is a single ccl_wave_step call;
nothing here computes on the data.
"""
from __future__ import annotations

import numpy as np

from . import (NEIGHBORHOOD, ccl_batch_create, ccl_batch_destroy, ccl_batch_grid,
               ccl_batch_result, ccl_batch_run, ccl_chunk_buffer, ccl_region_of, ccl_split_grid,
               ccl_split_range, ccl_wave_energy, ccl_wave_step, make_subrange, make_wave_params)

PITCH_ALIGN = 64  # elements; keeps every row start 256-byte aligned


def _round_up(v: int, a: int) -> int:
    return (v + a - 1) // a * a


def torch_dtype(dtype: str):
    import torch
    return {"f32": torch.float32, "f64": torch.float64, "bf16": torch.bfloat16,
            "f16": torch.float16}[dtype]


def alloc_buffer(region, device="cuda", fill=0.0, pitch_align=PITCH_ALIGN, dtype="f32"):
    """A torch tensor holding `region` (offset, range) row-major with a padded
    innermost pitch, and its ccl_chunk_buffer descriptor.  `dtype`: the
    element type ("f32", "f64", "bf16", "f16")."""
    import torch
    off, rng = region
    dims = len(rng)
    pitch_last = _round_up(int(rng[-1]), pitch_align)
    shape = tuple(int(r) for r in rng[:-1]) + (pitch_last,)
    t = torch.full(shape, float(fill), dtype=torch_dtype(dtype), device=device)
    b = ccl_chunk_buffer()
    b.base = t.data_ptr()
    b.region = make_subrange(off, rng)
    strides = t.stride()
    for d in range(dims):
        b.pitch[d] = int(strides[d])
    return t, b


def view_of(t, region, box):
    """Slice of buffer tensor `t` (holding `region`) covering global `box`."""
    (roff, _), (boff, brng) = region, box
    sl = tuple(slice(b - r, b - r + n) for r, b, n in zip(roff, boff, brng))
    return t[sl]


class ChunkedWave:
    """``nchunks`` chunks along ``split_dim`` (ccl_split_range), or, when
    ``grid`` gives a count per dimension, the block split of ccl_split_grid
    (``nchunks`` is then ignored).  ``dtype``: the fields' element type
    ("f32", "f64", "bf16", "f16"); scatter converts the host arrays to it
    (round to nearest even) and gather returns float64 for "f64", else
    float32."""

    def __init__(self, domain_offset, domain_shape, nchunks: int, r2: float, depth: int = 1,
                 tile_rows: int = 0, buffer_range=None, split_dim: int = 0, device="cuda",
                 fill=0.0, grid=None, dtype="f32"):
        self.dims = len(domain_shape)
        self.domain_offset = tuple(int(v) for v in domain_offset)
        self.domain_shape = tuple(int(v) for v in domain_shape)
        self.buffer_range = tuple(buffer_range) if buffer_range is not None else tuple(
            o + n for o, n in zip(self.domain_offset, self.domain_shape))
        self.depth = depth
        self.dtype = dtype
        self.params = make_wave_params(self.dims, r2, depth, tile_rows, dtype)
        if grid is not None:
            self.chunks = ccl_split_grid(self.domain_offset, self.domain_shape, grid)
        else:
            self.chunks = ccl_split_range(self.domain_offset, self.domain_shape, nchunks,
                                          split_dim)
        nchunks = len(self.chunks)
        self.nchunks = nchunks
        ext = (depth,) * self.dims
        self.regions = [ccl_region_of(c, NEIGHBORHOOD, ext, self.buffer_range).box()
                        for c in self.chunks]
        nbuf = 4 if depth > 1 else 2
        self.tensors = {}
        arrays = [(ccl_chunk_buffer * nchunks)() for _ in range(4)]
        for k, reg in enumerate(self.regions):
            for which in range(nbuf):
                t, b = alloc_buffer(reg, device=device, fill=fill, dtype=dtype)
                arrays[which][k] = b
                self.tensors[b.base] = (t, reg)
        self.u_prev, self.u_cur, self.w_prev, self.w_cur = arrays
        if nbuf == 2:
            self.w_prev = self.w_cur = None
        self.r2 = float(r2)
        self.n = 0  # leapfrog steps taken since the state was set

    def chunk_box(self, k):
        return self.chunks[k].box()

    def _local(self, box):
        (o, n) = box
        return tuple(slice(a - d, a - d + m) for a, d, m in zip(o, self.domain_offset, n))

    def scatter(self, u_prev, u_cur):
        """Copy host arrays of the domain's shape into every chunk's own cells."""
        import torch
        for k in range(self.nchunks):
            box = self.chunk_box(k)
            for arr, host in ((self.u_prev, u_prev), (self.u_cur, u_cur)):
                t, reg = self.tensors[arr[k].base]
                host_dt = np.float64 if self.dtype == "f64" else np.float32
                src = torch.from_numpy(np.ascontiguousarray(host[self._local(box)],
                                                            dtype=host_dt))
                view_of(t, reg, box).copy_(src, non_blocking=False)

    def gather(self, which="cur"):
        import torch
        arr = self.u_cur if which == "cur" else self.u_prev
        host_dt = np.float64 if self.dtype == "f64" else np.float32
        out = np.empty(self.domain_shape, dtype=host_dt)
        for k in range(self.nchunks):
            box = self.chunk_box(k)
            t, reg = self.tensors[arr[k].base]
            v = view_of(t, reg, box)
            if v.dtype in (torch.bfloat16, torch.float16):
                v = v.float()  # exact widening
            out[self._local(box)] = v.cpu().numpy()
        return out

    def gather_device(self, which="cur"):
        """The domain's cells of u^n ("cur") or u^{n-1} ("prev") copied into
        one contiguous device tensor of the element type."""
        import torch
        arr = self.u_cur if which == "cur" else self.u_prev
        first = self.tensors[arr[0].base][0]
        out = torch.empty(self.domain_shape, dtype=first.dtype, device=first.device)
        for k in range(self.nchunks):
            box = self.chunk_box(k)
            t, reg = self.tensors[arr[k].base]
            out[self._local(box)].copy_(view_of(t, reg, box))
        return out

    def energy(self, stream=None):
        """Discrete energy E^{n-1/2} of the state (u^{n-1}, u^n), computed on
        the device by ccl_wave_energy (u^n as the newer level)."""
        import torch
        a, b = self.gather_device("cur"), self.gather_device("prev")
        out = torch.zeros(1, dtype=torch.float64, device=a.device)
        ccl_wave_energy(self.domain_shape, [a.stride(d) for d in range(self.dims - 1)],
                        self.dtype, self.r2, a.data_ptr(), b.data_ptr(), out.data_ptr(), stream)
        return float(out.item())

    def gather_points(self, points, which="cur"):
        """Values at global indices `points` (list of tuples) of u_cur / u_prev."""
        arr = self.u_cur if which == "cur" else self.u_prev
        vals = []
        for p in points:
            for k in range(self.nchunks):
                (o, n) = self.chunk_box(k)
                if all(o[d] <= p[d] < o[d] + n[d] for d in range(self.dims)):
                    t, reg = self.tensors[arr[k].base]
                    idx = tuple(p[d] - reg[0][d] for d in range(self.dims))
                    vals.append(float(t[idx].item()))
                    break
            else:
                raise IndexError(p)
        return np.array(vals, dtype=np.float32)

    def step(self, nsteps: int, stream=None):
        ccl_wave_step(self.params, self.chunks, self.u_prev, self.u_cur, self.w_prev, self.w_cur,
                      nsteps, stream)
        self.n += int(nsteps)

    # Checkpoint / resume.  The leapfrog's whole state is its last two levels
    # (u^{n-1}, u^n) and the step count n: a run resumed from a checkpoint
    # continues exactly as the uninterrupted run (the halos are refilled by
    # the exchange before the next block).  With 16-bit storage the fields
    # are rounded at the end of every block of T steps, so a resumed run
    # matches the uninterrupted one when the checkpoint falls on a block
    # boundary of it.
    def save(self, path):
        """Writes the state to `path` (.npz): both levels of the domain as
        gathered (exact: 16-bit values widen exactly to float32), n, r2, the
        element type and the domain."""
        np.savez(path, u_prev=self.gather("prev"), u_cur=self.gather("cur"),
                 n=np.int64(self.n), r2=np.float64(self.r2), dtype=np.str_(self.dtype),
                 domain_offset=np.array(self.domain_offset, np.int64),
                 domain_shape=np.array(self.domain_shape, np.int64))

    def restore(self, path):
        """Sets the state from a checkpoint written by `save` for the same
        domain, element type and r2 (any chunking, depth or tile rows);
        returns n."""
        with np.load(path, allow_pickle=False) as f:
            if (tuple(f["domain_offset"].tolist()) != self.domain_offset or
                    tuple(f["domain_shape"].tolist()) != self.domain_shape):
                raise ValueError("checkpoint of another domain")
            if str(f["dtype"]) != self.dtype or float(f["r2"]) != self.r2:
                raise ValueError("checkpoint of another element type or r2")
            self.scatter(f["u_prev"], f["u_cur"])
            self.n = int(f["n"])
        return self.n


class BatchedWaves:
    """Buffers (four per grid, pitched rows) and a ccl_batch over them.

    ``specs``: list of dicts with ny, nx, steps, r2, depth and optionally
    tile_rows.  With ``create=False`` only the buffers and the grid
    descriptors (``grids``) are made, for ccl_batch_run_static."""

    def __init__(self, specs, device="cuda", flags=0, fill=0.0, create=True):
        import torch
        self.specs = [dict(s) for s in specs]
        self.tensors = []
        self.grids = []
        for s in self.specs:
            pitch = _round_up(int(s["nx"]), PITCH_ALIGN)
            ts = [torch.full((int(s["ny"]), pitch), float(fill), dtype=torch.float32,
                             device=device) for _ in range(4)]
            g = ccl_batch_grid()
            g.ny, g.nx, g.pitch = int(s["ny"]), int(s["nx"]), pitch
            g.steps = int(s["steps"])
            g.temporal_depth = int(s.get("depth", 1))
            g.tile_rows = int(s.get("tile_rows", 0))
            g.r2 = float(s["r2"])
            for k in range(4):
                g.buf[k] = ts[k].data_ptr()
            self.tensors.append(ts)
            self.grids.append(g)
        self.handle = ccl_batch_create(self.grids, flags) if create else None

    def scatter(self, g, u_prev, u_cur):
        import torch
        nx = self.specs[g]["nx"]
        self.tensors[g][0][:, :nx].copy_(torch.from_numpy(np.ascontiguousarray(u_prev, np.float32)))
        self.tensors[g][1][:, :nx].copy_(torch.from_numpy(np.ascontiguousarray(u_cur, np.float32)))

    def run(self, stream=None):
        ccl_batch_run(self.handle, stream)

    def gather(self, g, which="cur"):
        p, c = ccl_batch_result(self.handle, g)
        nx = self.specs[g]["nx"]
        return self.tensors[g][c if which == "cur" else p][:, :nx].cpu().numpy()

    def close(self):
        if self.handle is not None:
            ccl_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
