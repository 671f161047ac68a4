"""MI355X tiled-sCOLA engine (arXiv:2003.04925): Python front end of libscola.so.

The simulation runs in hand-written HIP kernels behind the C ABI of include/scola.h; this
package only allocates device memory with torch, marshals arguments and exposes the
results as torch tensors on the GPU.  There is no CPU path.
"""
import ctypes
from dataclasses import dataclass

from . import _lib
from ._lib import (SCOLA_BATCHED, SCOLA_FP32, SCOLA_FP64, SCOLA_PER_TILE, FIXED_BITS,
                   STATIC_WORKSPACE_BYTES, ScolaError)

__all__ = ["Simulation", "DensityFunction", "CosmologyParams", "uniform_tiling",
           "particle_order", "schedule_table",
           "linear_power", "ScolaError", "SCOLA_FP32", "SCOLA_FP64", "SCOLA_BATCHED",
           "SCOLA_PER_TILE", "FIXED_BITS", "STATIC_WORKSPACE_BYTES"]


@dataclass
class CosmologyParams:
    """Flat LambdaCDM; defaults: Omega_m and sigma_8 of the benchmark workloads, the other
    values of the paper's Planck 2015 set (Sec. 4)."""
    Omega_m: float = 0.31
    Omega_b: float = 0.0486
    h: float = 0.6774
    n_s: float = 0.9667
    sigma8: float = 0.81
    T_cmb: float = 2.7255

    def c(self):
        return _lib.Cosmology(self.Omega_m, self.Omega_b, self.h, self.n_s, self.sigma8,
                              self.T_cmb)


def particle_order(M):
    """Storage slot (inside a box's particle range) of every lattice site, sites flattened
    in lattice order [i][j][k].  The library keeps a box's particles in 4 x 8 x 8 bricks
    (one thread block each); this is only the index map, for inspecting the workspace."""
    import numpy as np
    i, j, k = np.meshgrid(np.arange(M), np.arange(M), np.arange(M), indexing="ij")
    nb = M // 8
    brick = ((i // 4) * nb + j // 8) * nb + k // 8
    w = ((i % 4) * 8 + j % 8) * 8 + k % 8
    return (brick * 256 + w).ravel()


def uniform_tiling(Np, tiles_per_side, buffer):
    """List of (core_lo (3,), core_n, buffer) from the library's uniform tiling."""
    n = tiles_per_side ** 3
    arr = (_lib.Tile * n)()
    _lib.check(_lib.lib().scola_uniform_tiling(Np, tiles_per_side, buffer, arr, n))
    return [(tuple(t.core_lo), t.core_n, t.buffer) for t in arr]


def _config(L, Np, n_steps, a_i, a_f, precision, schedule, want_momenta, N_out,
            checkpoint_every=0, discretisation="modified", n_lpt=0.0, N_lpt=0, fda_order=0):
    prec = {"fp32": SCOLA_FP32, "fp64": SCOLA_FP64}[precision]
    sch = {"batched": SCOLA_BATCHED, "per_tile": SCOLA_PER_TILE}[schedule]
    disc = {"modified": _lib.SCOLA_MODIFIED, "standard": _lib.SCOLA_STANDARD}[discretisation]
    return _lib.make_config(L, Np, n_steps, a_i, a_f, prec, sch, 1 if want_momenta else 0,
                            N_out or 0, checkpoint_every, N_lpt=N_lpt or 0,
                            fda_order=fda_order or 0, n_lpt=n_lpt or 0.0, discretisation=disc)


def schedule_table(n_steps, a_i=0.05, a_f=1.0, cosmology=None, discretisation="modified",
                   n_lpt=0.0):
    """Host FP64 KDK scalar rows (see scola_schedule_table); no device needed."""
    import numpy as np
    cfg = _config(1.0, 8, n_steps, a_i, a_f, "fp64", "batched", False, 0,
                  discretisation=discretisation, n_lpt=n_lpt)
    cosmo = (cosmology or CosmologyParams()).c()
    out = np.zeros((n_steps + 1, 8))
    _lib.check(_lib.lib().scola_schedule_table(
        ctypes.byref(cfg), ctypes.byref(cosmo),
        out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n_steps + 1))
    return out


def linear_power(k, cosmology=None):
    """P_lin(k, a = 1) of the library (host FP64)."""
    import numpy as np
    k = np.ascontiguousarray(k, dtype=np.float64)
    out = np.zeros_like(k)
    cosmo = (cosmology or CosmologyParams()).c()
    _lib.check(_lib.lib().scola_linear_power(
        ctypes.byref(cosmo), k.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
        out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), k.size))
    return out


class Simulation:
    """A tiled-sCOLA run on one GPU (one plan + one workspace).

    tiles: list of (core_lo (3 ints), core_n, buffer) or (core_lo, core_n, buffer, a_f) with
    a per-tile final scale factor (0 = a_f); or use uniform_tiling().
    precision: "fp32" (state, Psi and meshes in FP32, positions formed in FP64) or "fp64".
    schedule: "batched" (all boxes per launch) or "per_tile" (box after box).
    discretisation: "modified" (App. B time factors with u = a^n_lpt) or "standard".
    fda_order: 2 (default), 4 or 6, the finite-difference order of every Laplacian and
    gradient (the reverse mode and the persistent step are built for order 2).
    N_lpt: LPT grid nodes per side (default Np; or a power-of-two divisor such as Np // 2):
    the white noise has N_lpt^3 entries (the reverse mode and tCOLA need N_lpt = Np).
    mesh: as in include/scola.h (only the default is implemented; other values raise
    ScolaError with SCOLA_EUNSUPPORTED).
    """

    def __init__(self, L, Np, tiles, n_steps, a_i=0.05, a_f=1.0, precision="fp32",
                 schedule="batched", want_momenta=False, N_out=None, cosmology=None,
                 device=None, checkpoint_every=0, discretisation="modified", n_lpt=0.0,
                 N_lpt=0, fda_order=0, mesh=0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("a HIP device is required (the engine has no CPU path)")
        self.torch = torch
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else device)
        torch.cuda.set_device(self.device)
        torch.cuda.init()
        self.L, self.Np, self.n_steps = float(L), int(Np), int(n_steps)
        self.N_out = int(N_out or Np)
        self.precision = precision
        self.real = torch.float64 if precision == "fp64" else torch.float32
        self.want_momenta = bool(want_momenta)
        self.tiles = [(tuple(int(c) for c in t[0]), int(t[1]), int(t[2])) for t in tiles]
        self.tile_a_f = [float(t[3]) if len(t) > 3 else 0.0 for t in tiles]
        self.checkpoint_every = int(checkpoint_every)
        self.ghosts = (int(fda_order) or 2) // 2
        self.N_lpt = int(N_lpt or Np)
        cfg = _config(L, Np, n_steps, a_i, a_f, precision, schedule, want_momenta, N_out,
                      checkpoint_every, discretisation, n_lpt, N_lpt, fda_order)
        cosmo = (cosmology or CosmologyParams()).c()
        arr = (_lib.Tile * len(self.tiles))()
        for i, (lo, n, b) in enumerate(self.tiles):
            arr[i].core_lo[:] = lo
            arr[i].core_n = n
            arr[i].buffer = b
            arr[i].mesh[:] = (int(mesh),) * 3
            arr[i].a_f = self.tile_a_f[i]
        plan = ctypes.c_void_p()
        _lib.check(_lib.lib().scola_plan_create(ctypes.byref(cfg), ctypes.byref(cosmo), arr,
                                                len(self.tiles), ctypes.byref(plan)))
        self._plan = plan
        lay = _lib.Layout()
        _lib.check(_lib.lib().scola_workspace_layout(plan, ctypes.byref(lay)))
        self.layout = lay
        self.workspace = torch.empty(lay.total + 256, dtype=torch.uint8, device=self.device)
        self._generation = 0          # forward() calls so far (see DensityFunction)
        shift = (-self.workspace.data_ptr()) % 256
        self._ws_off = shift
        self._ws = ctypes.c_void_p(self.workspace.data_ptr() + shift)

    def __del__(self):
        plan = getattr(self, "_plan", None)
        if plan is not None and plan.value:
            try:
                _lib.lib().scola_plan_destroy(plan)
            except Exception:
                pass
            self._plan = None

    # --- helpers ---------------------------------------------------------------------
    def _stream(self):
        return ctypes.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    @staticmethod
    def _subset(tile_subset):
        if tile_subset is None:
            return None, 0
        arr = (ctypes.c_int32 * len(tile_subset))(*[int(t) for t in tile_subset])
        return arr, len(tile_subset)

    def view(self, name):
        """torch view of one workspace array (see scola_layout)."""
        t = self.torch
        lay = self.layout
        P, G, H, N = lay.n_particles, lay.n_nodes, lay.n_padded, self.Np
        rb = 8 if self.precision == "fp64" else 4
        spec = {
            "psi1": (self.real, (3, P)), "psi2": (self.real, (3, P)),
            "x_res": (self.real, (3, P)), "p_res": (self.real, (3, P)),
            # mass mesh: int64 (FP64 plans) or unsigned 32-bit held in an int32 view (FP32)
            "rho": (t.int64 if self.precision == "fp64" else t.int32, (G,)),
            "work": (self.real, (G,)), "phi": (self.real, (H,)),
            "bc0": (t.float64, (H,)),
            # dropped per tile, near-limit count, then (FP32) mass found and deposits per tile
            "dropped": (t.int64, (3 * len(self.tiles) + 1,)),
            # per brick of 256 particles: packed cell extent of its last deposit
            "cells": (t.int32, (P // 256, 4)),
            "phi1": (t.float64, (self.N_lpt,) * 3), "phi2": (t.float64, (self.N_lpt,) * 3),
            "outgrid": (t.int64, (self.N_out,) * 3),
        }[name]
        dtype, shape = spec
        nbytes = 1
        for s in shape:
            nbytes *= s
        nbytes *= {t.float64: 8, t.float32: 4, t.int64: 8, t.int32: 4}[dtype] \
            if dtype != self.real else rb
        off = self._ws_off + getattr(lay, name)
        return self.workspace[off:off + nbytes].view(dtype).view(shape)

    def _ptr(self, x, dtype, shape):
        if x is None:
            return None
        assert x.is_cuda and x.dtype == dtype and x.is_contiguous(), (x.dtype, dtype)
        assert tuple(x.shape) == tuple(shape), (tuple(x.shape), shape)
        return ctypes.c_void_p(x.data_ptr())

    # --- the run ---------------------------------------------------------------------
    def mass_alarm(self):
        """(near_limit, wrapped) counts of the FP32 mass mesh since the last evolution (see
        scola_mass_alarm); raises ScolaError (SCOLA_EOVERFLOW) when a node's mass wrapped.
        Synchronises the current stream."""
        near = ctypes.c_int64()
        wrapped = ctypes.c_int64()
        _lib.check(_lib.lib().scola_mass_alarm(self._plan, self._ws, self._stream(),
                                               ctypes.byref(near), ctypes.byref(wrapped)))
        return near.value, wrapped.value

    def forward(self, white_noise, tile_subset=None, density=True, momenta=None, check=True):
        """Run set-up, evolution and outputs.  Returns dict(pos, mom, density).  With check
        (default), the FP32 mass alarm is read afterwards (one stream synchronisation) and
        a wrapped node mass raises ScolaError."""
        t = self.torch
        Np = self.Np
        momenta = self.want_momenta if momenta is None else momenta
        pos = t.empty((3, Np, Np, Np), dtype=self.real, device=self.device)
        mom = t.empty_like(pos) if momenta else None
        dens = (t.empty((self.N_out,) * 3, dtype=self.real, device=self.device)
                if density and tile_subset is None else None)
        sub, n = self._subset(tile_subset)
        _lib.check(_lib.lib().scola_forward(
            self._plan, self._ptr(white_noise, t.float64, (self.N_lpt,) * 3),
            self._ptr(pos, self.real, pos.shape), self._ptr(mom, self.real, pos.shape)
            if mom is not None else None,
            self._ptr(dens, self.real, (self.N_out,) * 3) if dens is not None else None,
            sub, n, self._ws, self._stream()))
        self._generation += 1
        if check and self.precision == "fp32":
            self.mass_alarm()
        return dict(pos=pos, mom=mom, density=dens)

    def forward_noalloc(self, white_noise, density=True, momenta=None):
        """forward() over all tiles through scola_forward_noalloc: the library's static
        device workspace instead of this object's (the outputs are still allocated here)."""
        t = self.torch
        Np = self.Np
        momenta = self.want_momenta if momenta is None else momenta
        pos = t.empty((3, Np, Np, Np), dtype=self.real, device=self.device)
        mom = t.empty_like(pos) if momenta else None
        dens = t.empty((self.N_out,) * 3, dtype=self.real, device=self.device) if density else None
        _lib.check(_lib.lib().scola_forward_noalloc(
            self._plan, self._ptr(white_noise, t.float64, (self.N_lpt,) * 3),
            self._ptr(pos, self.real, pos.shape),
            self._ptr(mom, self.real, pos.shape) if mom is not None else None,
            self._ptr(dens, self.real, (self.N_out,) * 3) if dens is not None else None,
            self._stream()))
        return dict(pos=pos, mom=mom, density=dens)

    def tcola_forward(self, white_noise, density=True, momenta=None, record=False):
        """Monolithic periodic tCOLA of the full box (scola_tcola_forward) with this
        Simulation's schedule and precision, in its own workspace (allocated on first use).
        Returns dict(pos, mom, density, record_delta, record_phi); with record, the density
        contrast and potential of every force evaluation, shape (n_force, Np, Np, Np)."""
        t = self.torch
        Np = self.Np
        momenta = self.want_momenta if momenta is None else momenta
        if getattr(self, "_tcola_ws", None) is None:
            n = ctypes.c_size_t()
            _lib.check(_lib.lib().scola_tcola_workspace_size(self._plan, ctypes.byref(n)))
            self._tcola_buf = t.empty(n.value + 256, dtype=t.uint8, device=self.device)
            shift = (-self._tcola_buf.data_ptr()) % 256
            self._tcola_ws = ctypes.c_void_p(self._tcola_buf.data_ptr() + shift)
        pos = t.empty((3, Np, Np, Np), dtype=self.real, device=self.device)
        mom = t.empty_like(pos) if momenta else None
        dens = t.empty((self.N_out,) * 3, dtype=self.real, device=self.device) if density else None
        n_force = self.n_steps + (1 if self.want_momenta else 0)
        rd = rp = None
        if record:
            rd = t.empty((n_force, Np, Np, Np), dtype=self.real, device=self.device)
            rp = t.empty_like(rd)
        _lib.check(_lib.lib().scola_tcola_forward(
            self._plan, self._ptr(white_noise, t.float64, (self.N_lpt,) * 3),
            self._ptr(pos, self.real, pos.shape),
            self._ptr(mom, self.real, pos.shape) if mom is not None else None,
            self._ptr(dens, self.real, (self.N_out,) * 3) if dens is not None else None,
            self._ptr(rd, self.real, rd.shape) if rd is not None else None,
            self._ptr(rp, self.real, rp.shape) if rp is not None else None,
            self._tcola_ws, self._stream()))
        return dict(pos=pos, mom=mom, density=dens, record_delta=rd, record_phi=rp)

    def backward(self, grad_density):
        """d loss / d white noise (float64, [Np]^3) for d loss / d density (plan dtype,
        [N_out]^3); needs checkpoint_every > 0 and a preceding forward()."""
        t = self.torch
        grad_w = t.empty((self.N_lpt,) * 3, dtype=t.float64, device=self.device)
        _lib.check(_lib.lib().scola_backward(
            self._plan, self._ptr(grad_density.contiguous(), self.real, (self.N_out,) * 3),
            self._ptr(grad_w, t.float64, grad_w.shape), self._ws, self._stream()))
        return grad_w

    def setup(self, white_noise):
        t = self.torch
        _lib.check(_lib.lib().scola_setup(
            self._plan, self._ptr(white_noise, t.float64, (self.N_lpt,) * 3), self._ws,
            self._stream()))

    def evolve(self, tile_subset=None):
        sub, n = self._subset(tile_subset)
        _lib.check(_lib.lib().scola_evolve(self._plan, sub, n, self._ws, self._stream()))

    def evolve_overrides(self, delta=None, phi=None):
        """scola_evolve_overrides: the evolution with the density contrast and/or boundary
        potential of every force evaluation taken from full-box fields (n_force, Np, Np, Np)
        in the plan dtype, e.g. the record of tcola_forward (Sec. 4.3 consistency tests)."""
        n_force = self.n_steps + (1 if self.want_momenta else 0)
        shp = (n_force, self.Np, self.Np, self.Np)
        _lib.check(_lib.lib().scola_evolve_overrides(
            self._plan, self._ptr(delta, self.real, shp), self._ptr(phi, self.real, shp),
            self._ws, self._stream()))

    def output(self, pos=None, mom=None, density=None, tile_subset=None):
        sub, n = self._subset(tile_subset)
        shp = (3, self.Np, self.Np, self.Np)
        _lib.check(_lib.lib().scola_output(
            self._plan, self._ptr(pos, self.real, shp), self._ptr(mom, self.real, shp),
            self._ptr(density, self.real, (self.N_out,) * 3), sub, n, self._ws,
            self._stream()))

    def op_deposit(self, D1, D2):
        _lib.check(_lib.lib().scola_op_deposit(self._plan, D1, D2, self._ws, self._stream()))

    def op_poisson(self, D1_bc):
        _lib.check(_lib.lib().scola_op_poisson(self._plan, D1_bc, self._ws, self._stream()))

    def op_step(self, beta, alpha, D1, D2, D1n, D2n, deposit=True):
        _lib.check(_lib.lib().scola_op_step(self._plan, beta, alpha, D1, D2, D1n, D2n,
                                            1 if deposit else 0, self._ws, self._stream()))

    def op_final_kick(self, beta, D1, D2, c1, c2):
        _lib.check(_lib.lib().scola_op_final_kick(self._plan, beta, D1, D2, c1, c2, self._ws,
                                                  self._stream()))

    def step_table(self):
        import numpy as np
        out = np.zeros((self.n_steps + 1, 8))
        _lib.check(_lib.lib().scola_step_table(
            self._plan, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), self.n_steps + 1))
        return out

    def set_graph(self, enable):
        """Replay the batched evolution as a captured hipGraph (default) or run it eagerly."""
        _lib.check(_lib.lib().scola_plan_set_graph(self._plan, 1 if enable else 0))

    def set_persistent(self, enable):
        """One persistent cooperative launch per KDK step (scola_plan_set_persistent)."""
        _lib.check(_lib.lib().scola_plan_set_persistent(self._plan, 1 if enable else 0))

    def persistent(self):
        """dict(enabled, grid, barrier_failures) of the persistent step schedule."""
        e, g, f = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _lib.check(_lib.lib().scola_plan_persistent(self._plan, self._stream(), ctypes.byref(e),
                                                    ctypes.byref(g), ctypes.byref(f)))
        return dict(enabled=bool(e.value), grid=g.value, barrier_failures=f.value)

    def tune(self, reps=5):
        """Autotune the launch schedule on this workspace (after setup); returns it."""
        _lib.check(_lib.lib().scola_plan_tune(self._plan, self._ws, self._stream(), reps))
        return self.schedule()

    @property
    def groups(self):
        """Concurrent box groups of the batched evolution (1, 2 or 4)."""
        g = ctypes.c_int32()
        _lib.check(_lib.lib().scola_plan_concurrency(self._plan, ctypes.byref(g)))
        return g.value

    @groups.setter
    def groups(self, value):
        _lib.check(_lib.lib().scola_plan_set_concurrency(self._plan, int(value)))

    def schedule(self):
        """{M: {"waves_per_simd", "xcd_remap_particles", "xcd_remap_mesh"}} per box size."""
        n = ctypes.c_int32()
        _lib.check(_lib.lib().scola_plan_schedule(self._plan, None, 0, ctypes.byref(n)))
        arr = (_lib.ClassSchedule * n.value)()
        _lib.check(_lib.lib().scola_plan_schedule(self._plan, arr, n.value, ctypes.byref(n)))
        return {int(c.M): {"waves_per_simd": int(c.waves_per_simd),
                           "xcd_remap_particles": int(c.xcd_remap_particles),
                           "xcd_remap_mesh": int(c.xcd_remap_mesh)} for c in arr}

    def set_schedule(self, schedule):
        """schedule: as returned by schedule(), for every box size of the plan."""
        sizes = sorted(self.schedule())
        arr = (_lib.ClassSchedule * len(sizes))()
        for i, M in enumerate(sizes):
            d = schedule[M]
            arr[i] = _lib.ClassSchedule(M, d["waves_per_simd"], d["xcd_remap_particles"],
                                        d["xcd_remap_mesh"])
        _lib.check(_lib.lib().scola_plan_set_schedule(self._plan, arr, len(sizes)))

    def info(self):
        nt = ctypes.c_int32()
        np_ = ctypes.c_int64()
        r = ctypes.c_double()
        p = ctypes.c_double()
        _lib.check(_lib.lib().scola_plan_info(self._plan, ctypes.byref(nt), ctypes.byref(np_),
                                              ctypes.byref(r), ctypes.byref(p)))
        return dict(n_tiles=nt.value, n_particles=np_.value, r=r.value, p=p.value)

    def box_particles(self, arr, t):
        """Particle array [..., P] (workspace order) -> box t's sites in lattice order,
        shape [..., M, M, M]."""
        po, M, _, _ = self.box_slices()[t]
        return arr[..., po + particle_order(M)].reshape(arr.shape[:-1] + (M, M, M))

    def box_slices(self):
        """Per tile: (particle offset, M, interior-node offset, padded-node offset)."""
        out = []
        P = G = H = 0
        for lo, n, b in self.tiles:
            M = n + 2 * b
            out.append((P, M, G, H))
            P += M ** 3
            G += (M - 1) ** 3
            H += (M + 1 + 2 * self.ghosts) ** 3
        return out


class DensityFunction:
    """torch.autograd.Function: white noise (float64) -> output density (plan dtype).

    backward() runs the library's reverse mode (scola_backward), i.e. the hand-written
    adjoint of the whole chain, and returns d loss / d white noise."""

    @staticmethod
    def apply(sim, white_noise):
        return _density_fn().apply(white_noise, sim)


_FN = None


def _density_fn():
    global _FN
    if _FN is None:
        import torch

        class _Density(torch.autograd.Function):
            @staticmethod
            def forward(ctx, w, sim):
                ctx.sim = sim
                out = sim.forward(w, density=True)["density"]
                ctx.generation = sim._generation
                return out

            @staticmethod
            def backward(ctx, grad_out):
                # the library keeps one forward state per workspace: a later forward on the
                # same Simulation has replaced the trajectory this graph was built from
                if ctx.sim._generation != ctx.generation:
                    raise RuntimeError(
                        "DensityFunction.backward: the Simulation has run another forward "
                        "since this output was computed; its reverse mode would belong to "
                        "that later forward (use one Simulation per differentiated output)")
                return ctx.sim.backward(grad_out.to(ctx.sim.real)), None

        _FN = _Density
    return _FN
