"""MI355X-native steady-state memristor-crossbar (MCA) solver.

The solver is libmca.so (HIP kernels for gfx950 behind the C ABI of
include/mca.h).  This package is its Python binding: ``binding`` mirrors the
C entry points name for name, and :class:`Plan` bundles a plan with the torch
buffers (device memory) it needs.  ``synth`` draws seeded synthetic crossbars.
"""

from __future__ import annotations

from . import binding, synth
from .binding import (MCA_DEVICE_LINEAR, MCA_DEVICE_SINH, MCA_FLAG_INITIAL_GUESS,
                      MCA_PREC_BF16, MCA_PREC_BF16X3, MCA_PREC_FP32, MCA_PREC_FP64, MCA_PRECOND_LITERAL,
                      MCA_PRECOND_NONE, MCA_PRECOND_PERMODE, MCAError, mca_geometry,
                      mca_options, mca_stats, options)

__all__ = ["Plan", "Batch", "binding", "synth", "options", "MCAError", "mca_geometry", "mca_options",
           "mca_stats"]


class Plan:
    """A crossbar geometry's plan, uploaded to the current GPU.

    Holds the host plan handle and the device block of its eigenbases.  All
    array arguments are float64 torch tensors on the same GPU.
    """

    def __init__(self, geom, device="cuda"):
        import torch
        self.geom = geom
        self.m, self.n = int(geom.m), int(geom.n)
        self.device = torch.device(device)
        self.handle = binding.mca_plan_create(binding.geometry_from(geom))
        nbytes = binding.mca_plan_device_bytes(self.handle)
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        binding.mca_plan_upload(self.handle, self.buf)
        self._ws = None
        self._ws_key = None

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                binding.mca_plan_destroy(h)
            except Exception:   # interpreter shutdown: the library may be gone
                pass
            self.handle = None

    def _zeros(self):
        import torch
        return torch.zeros((self.m, self.n), dtype=torch.float64, device=self.device)

    def residual(self, g_dev, v_in, v_t, v_b):
        f_t, f_b, d = self._zeros(), self._zeros(), self._zeros()
        binding.mca_residual(self.handle, self.m, self.n, g_dev, v_in, v_t, v_b, f_t, f_b, d)
        return f_t, f_b, d

    def jacobian_apply(self, d, x_t, x_b):
        y_t, y_b = self._zeros(), self._zeros()
        binding.mca_jacobian_apply(self.handle, self.m, self.n, d, x_t, x_b, y_t, y_b)
        return y_t, y_b

    def precond_workspace(self, form, precision=MCA_PREC_FP64):
        import torch
        nbytes = binding.mca_precond_workspace_bytes(self.handle, form, precision)
        return torch.empty(nbytes, dtype=torch.uint8, device=self.device)

    def precond_apply(self, a1, a2, r_t, r_b, form=MCA_PRECOND_LITERAL,
                      precision=MCA_PREC_FP64, ws=None):
        z_t, z_b = self._zeros(), self._zeros()
        if ws is None:
            ws = self.precond_workspace(form, precision)
        binding.mca_precond_apply(self.handle, self.m, self.n, form, precision, a1, a2,
                                  r_t, r_b, z_t, z_b, ws)
        return z_t, z_b

    def workspace(self, opts=None):
        import torch
        nbytes = binding.mca_workspace_bytes(self.handle, opts)
        key = nbytes
        if self._ws is None or self._ws_key != key:
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self._ws_key = key
        return self._ws

    def solve(self, g_dev, v_in, opts=None, guess=None, out=None, check=True):
        """(v_t, v_b, status, stats) of the steady state."""
        if opts is None:
            opts = options()
        if out is None:
            v_t, v_b = self._zeros(), self._zeros()
        else:
            v_t, v_b = out
        if guess is not None:
            v_t.copy_(guess[0])
            v_b.copy_(guess[1])
            opts = mca_options.from_buffer_copy(opts)
            opts.flags |= MCA_FLAG_INITIAL_GUESS
        ws = self.workspace(opts)
        status, stats = binding.mca_solve(self.handle, self.m, self.n, g_dev, v_in, v_t, v_b,
                                          opts, ws, check=check)
        return v_t, v_b, status, stats


class Batch:
    """Many crossbars (sizes may differ) solved together on the current GPU.

    Arrays are concatenated float64 GPU tensors: crossbar b's m x n arrays at
    ``cross[b]:cross[b+1]``, its drives at ``rows[b]:rows[b+1]``.
    """

    def __init__(self, geoms, device="cuda"):
        import torch
        self.geoms = list(geoms)
        self.count = len(self.geoms)
        self.device = torch.device(device)
        self.handle = binding.mca_batch_create([binding.geometry_from(g) for g in self.geoms])
        self.cross, self.rows = binding.mca_batch_offsets(self.handle, self.count)
        nbytes = binding.mca_batch_device_bytes(self.handle)
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        binding.mca_batch_upload(self.handle, self.buf)
        self._ws = None
        self._ws_key = None

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                binding.mca_batch_destroy(h)
            except Exception:   # interpreter shutdown: the library may be gone
                pass
            self.handle = None

    @property
    def product_tile(self):
        """Tile edge (64 or 128) of the batch's grouped eigenbasis products."""
        return binding.mca_batch_product_tile(self.handle)

    @property
    def total(self):
        return int(self.cross[-1])

    def concat(self, arrays):
        """One contiguous float64 GPU tensor from per-crossbar arrays."""
        import torch
        return torch.cat([torch.as_tensor(a, dtype=torch.float64).reshape(-1) for a in arrays]).to(
            self.device).contiguous()

    def split(self, flat):
        """Per-crossbar (m, n) views of a concatenated array."""
        return [flat[int(self.cross[b]):int(self.cross[b + 1])].view(self.geoms[b].m, self.geoms[b].n)
                for b in range(self.count)]

    def workspace(self, opts):
        import torch
        nbytes = binding.mca_batch_workspace_bytes(self.handle, opts)
        if nbytes == 0:
            raise MCAError(binding.MCA_ERR_INVALID_ARG, "mca_batch_workspace_bytes")
        if self._ws is None or self._ws_key != nbytes:
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self._ws_key = nbytes
        return self._ws

    def solve(self, g_dev, v_in, opts=None, guess=None, out=None, check=True, ws=None):
        """(v_t, v_b, status, [stats]) over the concatenated arrays.  ws: optional
        workspace tensor (at least mca_batch_workspace_bytes) shared between batches."""
        import torch
        if opts is None:
            opts = options(precond=MCA_PRECOND_PERMODE, precision=MCA_PREC_BF16X3)
        if out is None:
            v_t = torch.zeros(self.total, dtype=torch.float64, device=self.device)
            v_b = torch.zeros(self.total, dtype=torch.float64, device=self.device)
        else:
            v_t, v_b = out
        if guess is not None:
            v_t.copy_(guess[0])
            v_b.copy_(guess[1])
            opts = mca_options.from_buffer_copy(opts)
            opts.flags |= MCA_FLAG_INITIAL_GUESS
        if ws is None:
            ws = self.workspace(opts)
        status, stats = binding.mca_solve_batched(self.handle, self.count, self.total,
                                                  int(self.rows[-1]), g_dev, v_in, v_t, v_b,
                                                  opts, ws, check=check)
        return v_t, v_b, status, stats
