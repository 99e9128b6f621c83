"""Device-side driver of one solver instance: PyTorch provides the device
buffer and the stream; every computation runs in libpflbm's kernels."""
import ctypes
import functools

import numpy as np
import torch

from . import pflbm as P


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Solver:
    """One coupled PF-LB state on the current CUDA (HIP) device.

    params: workload dict (see workloads.base_params); precision: "fp64",
    "fp32", "mixed_fp16" or "mixed_bf16"; state: an optional caller-owned
    uint8 device tensor of at least pflbm_state_bytes bytes to hold the
    state (allocated here otherwise); stream: the torch stream the library
    launches on (default: the current one). Every method runs with that
    stream current, so the tensors it allocates and returns belong to it;
    as for any torch side stream, a caller that uses a returned tensor on
    another stream, or passes in one produced on another stream, orders the
    two streams itself."""

    def __init__(self, params, precision="fp64", check_interval=0, zblock=0, device=None,
                 stream=None, tile="auto", state=None):
        if not torch.cuda.is_available():
            raise RuntimeError("libpflbm needs a GPU; none is visible")
        self.d = dict(params)
        self.precision = precision
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.p = P.make_params(self.d, precision, check_interval, zblock, tile)
        self.L = P.lib()
        nb = ctypes.c_size_t()
        self._check(self.L.pflbm_state_bytes(ctypes.byref(self.p), ctypes.byref(nb)), None)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        if state is None:
            with torch.cuda.stream(self.stream):
                state = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        elif state.dtype != torch.uint8 or not state.is_contiguous() or state.device != self.device:
            raise ValueError("state must be a contiguous uint8 tensor on %s" % self.device)
        self.state = state
        h = ctypes.c_void_p()
        self._check(self.L.pflbm_create(ctypes.byref(self.p), ctypes.c_void_p(self.stream.cuda_stream),
                                        _ptr(self.state), ctypes.c_size_t(self.state.numel()), ctypes.byref(h)),
                    None)
        self.h = h
        self.dim = 2 if self.d["lattice"] == "D2Q9_D2Q5" else 3
        self.shape = (int(self.d["nz"]), int(self.d["ny"]), int(self.d["nx"]))
        self.Qg, self.Qh = {"D2Q9_D2Q5": (9, 5), "D3Q19_D3Q7": (19, 7), "D3Q27_D3Q7": (27, 7)}[self.d["lattice"]]

    def _check(self, st, h):
        if st != P.PFLBM_OK:
            msg = self.L.pflbm_last_error(h).decode() if h else ""
            raise P.PflbmError(st, msg)

    def close(self):
        if getattr(self, "h", None):
            self.L.pflbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, a, shape):
        if a is None:
            return None
        t = torch.as_tensor(np.asarray(a) if not torch.is_tensor(a) else a)
        t = t.to(device=self.device, dtype=torch.float64).contiguous()
        if tuple(t.shape) != tuple(shape):
            t = t.reshape(shape)
        return t

    def init(self, phi0, u0=None, p0=None):
        phi = self._dev(phi0, self.shape)
        u = self._dev(u0, (self.dim,) + self.shape)
        pr = self._dev(p0, self.shape)
        self._keep = (phi, u, pr)   # alive until the stream has consumed them
        self._check(self.L.pflbm_init(self.h, _ptr(phi), _ptr(u), _ptr(pr)), self.h)

    def step(self, n=1):
        self._check(self.L.pflbm_step(self.h, int(n)), self.h)

    def run(self, nsteps, every, log, centre=None, R=0.0):
        """Advance nsteps, writing the float64 diagnostics of pflbm_volume as
        one JSON line (step, V_phi, V_count, sum_phi, phi_min, phi_max, umax,
        and with a centre the Laplace pressure jump dp = p_in - p_out) to log
        (a path, appended to, or a text file) at the start and after every
        `every` steps and the last one."""
        import json
        f = open(log, "a") if isinstance(log, (str, bytes)) or hasattr(log, "__fspath__") else log
        try:
            done = 0

            def write():
                v = self.volume(centre, R)
                rec = {"step": self.step_count()}
                rec.update({k: v[k] for k in ("V_phi", "V_count", "sum_phi", "phi_min", "phi_max", "umax")})
                if centre is not None:
                    rec["dp"] = v["p_in"] - v["p_out"]
                f.write(json.dumps(rec) + "\n")
            write()
            while done < nsteps:
                n = min(int(every), nsteps - done) if every > 0 else nsteps - done
                self.step(n)
                done += n
                write()
            f.flush()
        finally:
            if f is not log:
                f.close()

    def fields(self):
        phi = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        u = torch.empty((self.dim,) + self.shape, dtype=torch.float64, device=self.device)
        p = torch.empty_like(phi)
        rho = torch.empty_like(phi)
        self._check(self.L.pflbm_fields(self.h, _ptr(phi), _ptr(u), _ptr(p), _ptr(rho)), self.h)
        return phi, u, p, rho

    def volume(self, centre=None, R=0.0):
        out = P.pflbm_diag()
        c = (ctypes.c_double * 3)(*(list(centre) + [0.0] * (3 - len(centre)))) if centre is not None else None
        self._check(self.L.pflbm_volume(self.h, c, float(R), ctypes.byref(out)), self.h)
        return {k: getattr(out, k) for k, _ in P.pflbm_diag._fields_}

    def get_distributions(self):
        g = torch.empty((self.Qg,) + self.shape, dtype=torch.float64, device=self.device)
        h = torch.empty((self.Qh,) + self.shape, dtype=torch.float64, device=self.device)
        self._check(self.L.pflbm_get_distributions(self.h, _ptr(g), _ptr(h)), self.h)
        return g, h

    def step_record(self, f32=False):
        """One step; returns the state it started from, (g, h, pu) canonical,
        float64 or (f32) float32; pu is None for the models without (phi u)."""
        dt = torch.float32 if f32 else torch.float64
        g = torch.empty((self.Qg,) + self.shape, dtype=dt, device=self.device)
        h = torch.empty((self.Qh,) + self.shape, dtype=dt, device=self.device)
        pu = None
        if self.d.get("model", "AC") in ("CH", "L18", "L14"):
            pu = torch.empty((3,) + self.shape, dtype=dt, device=self.device)
        fn = self.L.pflbm_step_record_f32 if f32 else self.L.pflbm_step_record
        self._check(fn(self.h, _ptr(g), _ptr(h), _ptr(pu)), self.h)
        return g, h, pu

    def get_distributions_f32(self):
        g = torch.empty((self.Qg,) + self.shape, dtype=torch.float32, device=self.device)
        h = torch.empty((self.Qh,) + self.shape, dtype=torch.float32, device=self.device)
        self._check(self.L.pflbm_get_distributions_f32(self.h, _ptr(g), _ptr(h)), self.h)
        return g, h

    def set_distributions(self, g, h):
        g = self._dev(g, (self.Qg,) + self.shape)
        h = self._dev(h, (self.Qh,) + self.shape)
        self._keep = (g, h)
        self._check(self.L.pflbm_set_distributions(self.h, _ptr(g), _ptr(h)), self.h)

    def get_phiu(self):
        """(phi u) of the previous step, canonical float64 [3][z][y][x] (CH,
        Liang2018, Liang2014)."""
        pu = torch.empty((3,) + self.shape, dtype=torch.float64, device=self.device)
        self._check(self.L.pflbm_get_phiu(self.h, _ptr(pu)), self.h)
        return pu

    def set_phiu(self, pu):
        pu = self._dev(pu, (3,) + self.shape)
        self._keep = (pu,)
        self._check(self.L.pflbm_set_phiu(self.h, _ptr(pu)), self.h)

    def step_count(self):
        n = ctypes.c_longlong()
        self._check(self.L.pflbm_step_count(self.h, ctypes.byref(n)), self.h)
        return n.value

    def checkpoint_bytes(self):
        n = ctypes.c_size_t()
        self._check(self.L.pflbm_checkpoint_bytes(self.h, ctypes.byref(n)), self.h)
        return n.value

    def save_state(self, buf=None):
        if buf is None:
            buf = torch.empty(self.checkpoint_bytes(), dtype=torch.uint8, device=self.device)
        self._check(self.L.pflbm_save_state(self.h, _ptr(buf)), self.h)
        return buf

    def load_state(self, buf):
        self._check(self.L.pflbm_load_state(self.h, _ptr(buf)), self.h)

    # ---- discrete adjoint (every model)
    def adjoint_workspace(self):
        n = ctypes.c_size_t()
        self._check(self.L.pflbm_adjoint_workspace_bytes(self.h, ctypes.byref(n)), self.h)
        return torch.empty(n.value, dtype=torch.uint8, device=self.device)

    def adjoint_step(self, fwd_g, fwd_h, lam_g, lam_h, out_g, out_h, dparams, work):
        """lambda^n (out_g, out_h) from lambda^{n+1} (lam_g, lam_h) at the forward
        state (fwd_g, fwd_h); adds dL/d(sigma, M, W) into dparams (float64 [3])."""
        self._check(self.L.pflbm_adjoint_step(self.h, _ptr(fwd_g), _ptr(fwd_h), _ptr(lam_g),
                                              _ptr(lam_h), _ptr(out_g), _ptr(out_h),
                                              _ptr(dparams), _ptr(work)), self.h)

    def adjoint_step_pu(self, fwd_g, fwd_h, fwd_pu, lam_g, lam_h, lam_pu, out_g, out_h, out_pu, dparams,
                        work):
        """adjoint_step with the (phi u) state of the CH model
        (pflbm_adjoint_step_pu)."""
        self._check(self.L.pflbm_adjoint_step_pu(self.h, _ptr(fwd_g), _ptr(fwd_h), _ptr(fwd_pu), _ptr(lam_g),
                                                 _ptr(lam_h), _ptr(lam_pu), _ptr(out_g), _ptr(out_h),
                                                 _ptr(out_pu), _ptr(dparams), _ptr(work)), self.h)

    def adjoint_step_f32(self, fwd_g, fwd_h, lam_g, lam_h, out_g, out_h, dparams, work):
        """The float32 adjoint step of the AC model (float32 tensors; dparams
        float64)."""
        self._check(self.L.pflbm_adjoint_step_f32(self.h, _ptr(fwd_g), _ptr(fwd_h), _ptr(lam_g), _ptr(lam_h),
                                                  _ptr(out_g), _ptr(out_h), _ptr(dparams), _ptr(work)), self.h)

    def adjoint_step_pu_f32(self, fwd_g, fwd_h, fwd_pu, lam_g, lam_h, lam_pu, out_g, out_h, out_pu, dparams,
                            work):
        """The float32 adjoint step of the CH model, (phi u) included."""
        self._check(self.L.pflbm_adjoint_step_pu_f32(
            self.h, _ptr(fwd_g), _ptr(fwd_h), _ptr(fwd_pu), _ptr(lam_g), _ptr(lam_h), _ptr(lam_pu),
            _ptr(out_g), _ptr(out_h), _ptr(out_pu), _ptr(dparams), _ptr(work)), self.h)

    def adjoint_init_pu_f32(self, phi0, u0, p0, lam_g, lam_h, lam_pu, dparams, work):
        """float32 dL/dphi0 of the CH initialisation; adds its sigma and W terms
        into dparams (float64)."""
        phi = self._dev(phi0, self.shape)
        u = self._dev(u0, (self.dim,) + self.shape)
        pr = self._dev(p0, self.shape)
        out = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        self._check(self.L.pflbm_adjoint_init_pu_f32(self.h, _ptr(phi), _ptr(u), _ptr(pr), _ptr(lam_g), _ptr(lam_h),
                                                     _ptr(lam_pu), _ptr(out), _ptr(dparams), _ptr(work)), self.h)
        return out

    def adjoint_seed_phi_f32(self, dphi):
        dphi = torch.as_tensor(dphi, device=self.device).to(torch.float32).contiguous().reshape(self.shape)
        lam_g = torch.empty((self.Qg,) + self.shape, dtype=torch.float32, device=self.device)
        lam_h = torch.empty((self.Qh,) + self.shape, dtype=torch.float32, device=self.device)
        self._keep = (dphi,)
        self._check(self.L.pflbm_adjoint_seed_phi_f32(self.h, _ptr(dphi), _ptr(lam_g), _ptr(lam_h)), self.h)
        return lam_g, lam_h

    def adjoint_init_f32(self, phi0, u0, p0, lam_g, lam_h):
        phi = self._dev(phi0, self.shape)
        u = self._dev(u0, (self.dim,) + self.shape)
        pr = self._dev(p0, self.shape)
        out = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        self._check(self.L.pflbm_adjoint_init_f32(self.h, _ptr(phi), _ptr(u), _ptr(pr), _ptr(lam_g), _ptr(lam_h),
                                                  _ptr(out)), self.h)
        return out

    def adjoint_step_noalloc(self, fwd_g, fwd_h, lam_g, lam_h, out_g, out_h, dparams):
        """adjoint_step without a workspace (the library's own device scratch)."""
        self._check(self.L.pflbm_adjoint_step_noalloc(self.h, _ptr(fwd_g), _ptr(fwd_h), _ptr(lam_g),
                                                      _ptr(lam_h), _ptr(out_g), _ptr(out_h),
                                                      _ptr(dparams)), self.h)

    def adjoint_seed_phi(self, dphi):
        """(lambda_g, lambda_h) of a loss with gradient dphi with respect to the
        phase field of a state (pflbm_adjoint_seed_phi)."""
        dphi = self._dev(dphi, self.shape)
        lam_g = torch.empty((self.Qg,) + self.shape, dtype=torch.float64, device=self.device)
        lam_h = torch.empty((self.Qh,) + self.shape, dtype=torch.float64, device=self.device)
        self._keep = (dphi,)
        self._check(self.L.pflbm_adjoint_seed_phi(self.h, _ptr(dphi), _ptr(lam_g), _ptr(lam_h)), self.h)
        return lam_g, lam_h

    def adjoint_seed(self, fwd_h, dphi, dparams, work):
        """(lambda_g, lambda_h) of a loss with gradient dphi with respect to the
        phase field pflbm_fields returns for the state with h = fwd_h; adds the
        nonlocal correction's M and W terms into dparams (pflbm_adjoint_seed)."""
        dphi = self._dev(dphi, self.shape)
        lam_g = torch.empty((self.Qg,) + self.shape, dtype=torch.float64, device=self.device)
        lam_h = torch.empty((self.Qh,) + self.shape, dtype=torch.float64, device=self.device)
        self._keep = (dphi,)
        self._check(self.L.pflbm_adjoint_seed(self.h, _ptr(fwd_h), _ptr(dphi), _ptr(lam_g), _ptr(lam_h),
                                              _ptr(dparams), _ptr(work)), self.h)
        return lam_g, lam_h

    def adjoint_init(self, phi0, u0, p0, lam_g, lam_h):
        phi = self._dev(phi0, self.shape)
        u = self._dev(u0, (self.dim,) + self.shape)
        pr = self._dev(p0, self.shape)
        out = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        self._check(self.L.pflbm_adjoint_init(self.h, _ptr(phi), _ptr(u), _ptr(pr), _ptr(lam_g),
                                              _ptr(lam_h), _ptr(out)), self.h)
        return out

    def adjoint_init_pu(self, phi0, u0, p0, lam_g, lam_h, lam_pu, dparams, work):
        """dL/dphi0 of the initialisation with the (phi u) part; adds the sigma
        and W terms of the CH initialisation into dparams."""
        phi = self._dev(phi0, self.shape)
        u = self._dev(u0, (self.dim,) + self.shape)
        pr = self._dev(p0, self.shape)
        out = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        self._check(self.L.pflbm_adjoint_init_pu(self.h, _ptr(phi), _ptr(u), _ptr(pr), _ptr(lam_g),
                                                 _ptr(lam_h), _ptr(lam_pu), _ptr(out), _ptr(dparams),
                                                 _ptr(work)), self.h)
        return out


def _on_stream(fn):
    @functools.wraps(fn)
    def wrapped(self, *args, **kwargs):
        if self.stream == torch.cuda.current_stream(self.device):
            return fn(self, *args, **kwargs)
        with torch.cuda.stream(self.stream):
            return fn(self, *args, **kwargs)
    return wrapped


for _name, _fn in list(vars(Solver).items()):
    if callable(_fn) and not _name.startswith("_") and _name not in ("close", "step_count", "checkpoint_bytes"):
        setattr(Solver, _name, _on_stream(_fn))
del _name, _fn
