"""Python surface of the flame stepper: device memory and streams from torch,
every step of the computation in the HIP library (libflamefront.so)."""

import ctypes

import numpy as np
import torch

from . import native


def _dev_tensor(x, dtype, device):
    if isinstance(x, np.ndarray):
        x = torch.from_numpy(np.ascontiguousarray(x))
    return x.to(device=device, dtype=dtype).contiguous()


class FlameEnsemble:
    """A plan over one or more flames (possibly of different grids).

    descs: list of dicts with keys n1, n2 and optionally gamma, theta_pi, t0,
    dt, axis_scale, r0_law (1: the reference radius comes from a table given
    with set_r0_table), integrator (0 or "euler": integrating-factor Euler;
    1 or "rk2": integrating-factor Heun). The plan is bound to the current
    torch stream of `device`.
    """

    def __init__(self, descs, device="cuda", ws_fill=None):
        if not torch.cuda.is_available():
            raise RuntimeError("the flame stepper needs a ROCm GPU (torch.cuda is unavailable)")
        self.lib = native.load()
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.params = [dict(d) for d in descs]
        self.descs = [native.make_desc(**d) for d in self.params]
        self.states = []
        with torch.cuda.device(self.device):
            for d in self.descs:
                nb = native.state_bytes(d)
                self.states.append(torch.zeros(nb // 8, dtype=torch.complex64, device=self.device))
            ws_bytes = native.workspace_bytes(self.descs)
            self.ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=self.device)
            if ws_fill is not None:
                self.ws.fill_(int(ws_fill))
            off = (-self.ws.data_ptr()) % 256
            self.ws_ptr = self.ws.data_ptr() + off
            self.stream = torch.cuda.current_stream(self.device)
            arr = (native.FlameDesc * len(self.descs))(*self.descs)
            ptrs = (ctypes.c_void_p * len(self.states))(*[s.data_ptr() for s in self.states])
            plan = ctypes.c_void_p()
            native.check(self.lib.flame_init(arr, len(self.descs), ptrs, ctypes.c_void_p(self.ws_ptr),
                                             ws_bytes, ctypes.c_void_p(self.stream.cuda_stream),
                                             ctypes.byref(plan)))
        self.plan = plan

    # ------------------------------------------------------------ helpers
    def _check_flame(self, f):
        if not 0 <= f < len(self.descs):
            raise IndexError(f"flame index {f} out of range")

    def half_shape(self, f=0):
        d = self.descs[f]
        return (d.n1 // 2 - 1, d.n2 // 4)

    # ------------------------------------------------------------ state I/O
    def set_spectrum(self, half, n=0, flame=0):
        """Load the canonical half spectrum (complex64, shape (2K1+1, K2+1))."""
        self._check_flame(flame)
        h = _dev_tensor(half, torch.complex64, self.device)
        if tuple(h.shape) != self.half_shape(flame):
            raise ValueError(f"half spectrum has shape {tuple(h.shape)}, expected {self.half_shape(flame)}")
        native.check(self.lib.flame_set_spectrum(self.plan, flame, ctypes.c_void_p(h.data_ptr()), int(n)))
        self._keep = h

    def spectrum(self, flame=0):
        self._check_flame(flame)
        out = torch.empty(self.half_shape(flame), dtype=torch.complex64, device=self.device)
        native.check(self.lib.flame_get_spectrum(self.plan, flame, ctypes.c_void_p(out.data_ptr())))
        return out

    def set_phi(self, phi, n=0, flame=0):
        """Project a physical field (float32, n1 x n2) onto the retained box."""
        self._check_flame(flame)
        d = self.descs[flame]
        x = _dev_tensor(phi, torch.float32, self.device)
        if tuple(x.shape) != (d.n1, d.n2):
            raise ValueError(f"field has shape {tuple(x.shape)}, expected {(d.n1, d.n2)}")
        native.check(self.lib.flame_set_state(self.plan, flame, ctypes.c_void_p(x.data_ptr()), int(n)))
        self._keep = x

    def phi(self, flame=0):
        self._check_flame(flame)
        d = self.descs[flame]
        out = torch.empty((d.n1, d.n2), dtype=torch.float32, device=self.device)
        native.check(self.lib.flame_get_state(self.plan, flame, ctypes.c_void_p(out.data_ptr())))
        return out

    def state_modified(self, n, flame=-1):
        """The state buffer of `flame` (-1: of every flame) was written directly:
        set the step index to n and rebuild that flame's intermediates at the next step."""
        if flame != -1:
            self._check_flame(flame)
        native.check(self.lib.flame_state_modified(self.plan, int(flame), int(n)))

    @property
    def step_index(self):
        v = ctypes.c_int64()
        native.check(self.lib.flame_step_index(self.plan, ctypes.byref(v)))
        return v.value

    # ------------------------------------------------------------ stepping
    def step(self, nsteps=1):
        native.check(self.lib.flame_step(self.plan, int(nsteps)))

    def diagnostics(self, flame=0, out=None, dJ_dstate=None):
        """Mean radius, averaged velocity, area excess and finite flag (doubles);
        with dJ_dstate (a device tensor in the state layout) also the adjoint seed
        dJ/dPhi at the current state, written there."""
        self._check_flame(flame)
        buf = out if out is not None else torch.empty(4, dtype=torch.float64, device=self.device)
        seed = ctypes.c_void_p(dJ_dstate.data_ptr()) if dJ_dstate is not None else None
        native.check(self.lib.flame_diagnostics(self.plan, flame, ctypes.c_void_p(buf.data_ptr()), seed))
        if out is not None:
            return out
        v = buf.cpu().tolist()
        return {"mean_radius": v[0], "velocity": v[1], "area_excess": v[2], "finite": bool(v[3] == 1.0)}

    def check_finite(self, flame=0):
        """Averages in host memory (waits for the stream); raises FlameError with
        code FLAME_ERR_NONFINITE if the state holds non-finite values."""
        self._check_flame(flame)
        out = (ctypes.c_double * 4)()
        native.check(self.lib.flame_diagnostics_host(self.plan, flame, out))
        return {"mean_radius": out[0], "velocity": out[1], "area_excess": out[2], "finite": out[3] == 1.0}

    # ------------------------------------------------------------ adjoint
    def new_cotangent(self, flame=0):
        """Zeroed buffer in the state layout (for cotangents and saved states)."""
        return torch.zeros_like(self.states[flame])

    def adjoint_step(self, n, state_n, lam_in, lam_out, flame=0):
        """lam_out = (d Phi^{n+1} / d Phi^n)^T lam_in for the step taken from state_n."""
        self._check_flame(flame)
        native.check(self.lib.flame_adjoint_step(self.plan, flame, int(n), ctypes.c_void_p(state_n.data_ptr()),
                                                 ctypes.c_void_p(lam_in.data_ptr()),
                                                 ctypes.c_void_p(lam_out.data_ptr())))

    def area_gradient(self, n, state, lam_out, flame=0):
        """lam_out = dJ/dPhi of the area excess at `state` (step index n)."""
        self._check_flame(flame)
        native.check(self.lib.flame_area_gradient(self.plan, flame, int(n), ctypes.c_void_p(state.data_ptr()),
                                                  ctypes.c_void_p(lam_out.data_ptr())))

    def synthesize(self, spec, flame=0):
        """Grid field (float32, n1 x n2) of a spectrum in the state layout."""
        self._check_flame(flame)
        d = self.descs[flame]
        out = torch.empty((d.n1, d.n2), dtype=torch.float32, device=self.device)
        native.check(self.lib.flame_synthesize(self.plan, flame, ctypes.c_void_p(spec.data_ptr()),
                                               ctypes.c_void_p(out.data_ptr())))
        return out

    def set_points_per_thread(self, n1, n2, col_pts, row_pts):
        """Points per thread (8 or 16) of the step kernels for the grid n1 x n2."""
        native.check(self.lib.flame_set_points_per_thread(self.plan, int(n1), int(n2), int(col_pts), int(row_pts)))

    def points_per_thread(self, n1, n2):
        c, r = ctypes.c_int32(), ctypes.c_int32()
        native.check(self.lib.flame_get_points_per_thread(self.plan, int(n1), int(n2), ctypes.byref(c),
                                                          ctypes.byref(r)))
        return c.value, r.value

    def set_r0_table(self, table, flame=0):
        """Reference-radius table of a flame with r0_law = 1: a float64 tensor of
        shape (n, 3) on the plan's device, row n = (r0(t_n), int_{t_n}^{t_n+1} ds/r0,
        int ds/r0^2). The tensor is kept alive by this object."""
        self._check_flame(flame)
        if table.dtype != torch.float64 or table.dim() != 2 or table.shape[1] != 3 or table.device != self.device:
            raise ValueError("table must be a float64 (n, 3) tensor on the plan's device")
        table = table.contiguous()
        native.check(self.lib.flame_set_r0_table(self.plan, int(flame), ctypes.c_void_p(table.data_ptr()),
                                                 int(table.shape[0])))
        if not hasattr(self, "_r0_tables"):
            self._r0_tables = {}
        self._r0_tables[flame] = table

    def set_forcing(self, half, flame=0):
        """Forcing f~_k of Eq. (1) for a flame, taken by every later step: a
        canonical half spectrum (complex64, shape (2K1+1, K2+1), the layout of
        set_spectrum), or None for no forcing. The values are copied, on the
        plan's stream, into a state-layout buffer that this object keeps and
        the library reads; calling again between steps gives a forcing that
        varies in time."""
        self._check_flame(flame)
        if not hasattr(self, "_forcing"):
            self._forcing = {}
        if half is None:
            native.check(self.lib.flame_set_forcing(self.plan, int(flame), None))
            self._forcing.pop(flame, None)
            return
        with torch.cuda.stream(self.stream):
            h = _dev_tensor(half, torch.complex64, self.device)
            if tuple(h.shape) != self.half_shape(flame):
                raise ValueError(f"forcing has shape {tuple(h.shape)}, expected {self.half_shape(flame)}")
            buf = self._forcing.get(flame)
            if buf is None:
                d = self.descs[flame]
                # state layout [k2][k1 + n1/4]; the slot k1 = -n1/4 lies outside the box
                buf = torch.zeros((d.n2 // 4, d.n1 // 2), dtype=torch.complex64, device=self.device)
            buf[:, 1:].copy_(h.t())
        if flame not in self._forcing:
            native.check(self.lib.flame_set_forcing(self.plan, int(flame), ctypes.c_void_p(buf.data_ptr())))
            self._forcing[flame] = buf

    def set_product_grid(self, n1, n2, enable):
        """Form the quadratic term on 3*n1/4 theta rows (True) or on n1 rows (False)
        for the flames of grid n1 x n2; the results agree to rounding."""
        native.check(self.lib.flame_set_product_grid(self.plan, int(n1), int(n2), int(bool(enable))))

    def product_grid(self, n1, n2):
        v = ctypes.c_int32()
        native.check(self.lib.flame_get_product_grid(self.plan, int(n1), int(n2), ctypes.byref(v)))
        return bool(v.value)

    def set_streaming_stores(self, n1, n2, enable):
        """Write the step's intermediates of the flames of grid n1 x n2 with
        non-temporal stores: True or 1 both Q and W, 2 W only, 3 Q only; False
        or 0 plain stores. The results are identical."""
        native.check(self.lib.flame_set_streaming_stores(self.plan, int(n1), int(n2), int(enable)))

    def streaming_stores(self, n1, n2):
        """The store kind: 0 plain, 1 non-temporal Q and W, 2 W only, 3 Q only."""
        v = ctypes.c_int32()
        native.check(self.lib.flame_get_streaming_stores(self.plan, int(n1), int(n2), ctypes.byref(v)))
        return v.value

    def autotune(self, steps=20):
        """Time every grid, points-per-thread and store-kind choice per grid group and
        keep the fastest; the simulation state is unchanged. Returns the number of
        timed configurations."""
        tried = ctypes.c_int32()
        native.check(self.lib.flame_autotune(self.plan, int(steps), ctypes.byref(tried)))
        return tried.value

    def set_graph_steps(self, steps):
        """Step in hipGraphs of `steps` steps (0: direct launches)."""
        native.check(self.lib.flame_set_graph_steps(self.plan, int(steps)))

    def set_persistent(self, enable=True, workgroups=0, wait_limit_us=0):
        """Step every flame in one persistent (cooperative) launch per call, or,
        with set_graph_steps(k), in replays of a graph holding that launch for k
        steps (workgroups 0: all that fit; wait_limit_us 0: 2 s per wait)."""
        native.check(self.lib.flame_set_persistent(self.plan, int(bool(enable)), int(workgroups),
                                                   int(wait_limit_us)))

    def persistent(self):
        """(enabled, workgroups of the last persistent launch)."""
        on, wgs = ctypes.c_int32(0), ctypes.c_int32(0)
        native.check(self.lib.flame_get_persistent(self.plan, ctypes.byref(on), ctypes.byref(wgs)))
        return bool(on.value), wgs.value

    def timing_begin(self):
        native.check(self.lib.flame_timing_begin(self.plan))

    def timing_end(self):
        """Summed milliseconds and counts: row, column, diagnostics kernels, graph launches."""
        ms = (ctypes.c_double * 4)()
        cnt = (ctypes.c_int64 * 4)()
        native.check(self.lib.flame_timing_end(self.plan, ms, cnt))
        keys = ("row", "col", "diag", "graph")
        return {k: (ms[i], cnt[i]) for i, k in enumerate(keys)}

    def close(self):
        if getattr(self, "plan", None):
            native.check(self.lib.flame_destroy(self.plan))
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FlameSim(FlameEnsemble):
    """One flame: FlameSim(n1, n2, gamma=0.8, theta_pi=1.0, t0=200.0, dt=0.25)."""

    def __init__(self, n1, n2, device="cuda", ws_fill=None, **kw):
        super().__init__([dict(n1=n1, n2=n2, **kw)], device=device, ws_fill=ws_fill)


class _FlameArea(torch.autograd.Function):
    """J(phi0) = area excess after nsteps, with a checkpointed hand-written adjoint."""

    @staticmethod
    def forward(ctx, phi0, sim, nsteps, checkpoint_every, flame):
        sim.set_phi(phi0.detach(), n=0, flame=flame)
        checkpoints = []
        n = 0
        while n < nsteps:
            checkpoints.append((n, sim.states[flame].clone()))
            k = min(checkpoint_every, nsteps - n)
            sim.step(k)
            n += k
        final = sim.states[flame].clone()
        area = sim.diagnostics(flame)["area_excess"]
        ctx.sim, ctx.nsteps, ctx.every, ctx.flame = sim, nsteps, checkpoint_every, flame
        ctx.checkpoints, ctx.final = checkpoints, final
        return torch.tensor(area, dtype=torch.float64, device=phi0.device)

    @staticmethod
    def backward(ctx, grad_out):
        sim, f = ctx.sim, ctx.flame
        lam = sim.new_cotangent(f)
        sim.area_gradient(ctx.nsteps, ctx.final, lam, flame=f)
        for n0, saved in reversed(ctx.checkpoints):
            k = min(ctx.every, ctx.nsteps - n0)
            # recompute the states n0 .. n0+k-1 of this segment from its checkpoint
            ring = [saved]
            sim.states[f].copy_(saved)
            sim.state_modified(n0)
            for _ in range(1, k):
                sim.step(1)
                ring.append(sim.states[f].clone())
            for i in reversed(range(k)):
                sim.adjoint_step(n0 + i, ring[i], lam, lam, flame=f)
        grad = sim.synthesize(lam, flame=f)
        return grad * grad_out.to(grad.dtype), None, None, None, None


def flame_area(phi0, sim, nsteps, checkpoint_every=50, flame=0):
    """Area excess J after nsteps from the physical initial field phi0 (float32,
    n1 x n2, on the sim's device), differentiable with respect to phi0 through
    the library's adjoint (states are checkpointed every `checkpoint_every`
    steps and recomputed in the backward pass). The sim's state is overwritten."""
    return _FlameArea.apply(phi0, sim, int(nsteps), int(checkpoint_every), int(flame))


class CircleBatch:
    """A batch of circular flames of one grid (the one-dimensional form of
    Eq. (1)): CircleBatch(n, count, gamma=0.8, seg=1.0, t0=200.0, dt=0.25).
    The spectra live in one complex64 tensor of shape (count, n/4) on the
    device (k = 0 .. n/4 - 1); every step runs in the HIP library."""

    def __init__(self, n, count, device="cuda", **kw):
        if not torch.cuda.is_available():
            raise RuntimeError("the flame stepper needs a ROCm GPU (torch.cuda is unavailable)")
        self.lib = native.load()
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.desc = native.make_circle_desc(n, **kw)
        nb = ctypes.c_size_t()
        native.check(self.lib.flame_circle_state_bytes(ctypes.byref(self.desc), ctypes.byref(nb)))
        self.count = int(count)
        self.states = torch.zeros((self.count, nb.value // 8), dtype=torch.complex64, device=self.device)
        self.n = 0

    def _stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def set_spectra(self, spectra, n=0):
        """Load the spectra (count x n/4 complex, k = 0 .. n/4 - 1) at step index n."""
        s = _dev_tensor(spectra, torch.complex64, self.device)
        if tuple(s.shape) != tuple(self.states.shape):
            raise ValueError(f"spectra have shape {tuple(s.shape)}, expected {tuple(self.states.shape)}")
        self.states.copy_(s)
        self.n = int(n)

    def step(self, nsteps=1):
        native.check(self.lib.flame_circle_step(ctypes.byref(self.desc), self.count,
                                                ctypes.c_void_p(self.states.data_ptr()), self.n, int(nsteps),
                                                self._stream()))
        self.n += int(nsteps)

    def diagnostics(self, out=None):
        """(count, 4) float64 tensor: mean radius, <Phi_t>, length excess, finite flag."""
        buf = out if out is not None else torch.empty((self.count, 4), dtype=torch.float64, device=self.device)
        native.check(self.lib.flame_circle_diagnostics(ctypes.byref(self.desc), self.count,
                                                       ctypes.c_void_p(self.states.data_ptr()), self.n,
                                                       ctypes.c_void_p(buf.data_ptr()), self._stream()))
        return buf
