"""Python binding of the WLS-ENO C-ABI (marshalling only).

Every numerical step runs in the HIP kernels of ``libwlseno.so``; this module
passes pointers, sizes and torch's current HIP stream, and turns status codes
into exceptions.  Device arrays are ``torch.float64`` tensors on the GPU.
"""

from __future__ import annotations

import ctypes as C

import numpy as np

from . import _native as N


class WLSENOError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{N.STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


class WLSENO:
    """One context: a mesh, its stencils and the device data of one parameter set."""

    def __init__(self, device: int = 0):
        self._lib = N.load()
        h = C.c_void_p()
        st = self._lib.wlseno_create(int(device), None, C.byref(h))
        if st != N.WLSENO_OK:
            raise WLSENOError(st, self._lib.wlseno_last_error(None).decode())
        self._h = h
        self.device = int(device)
        self.dim = None
        self.n_cell = None

    def close(self):
        if getattr(self, "_h", None):
            self._lib.wlseno_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != N.WLSENO_OK:
            raise WLSENOError(st, self._lib.wlseno_last_error(self._h).decode())

    def _sync_stream(self):
        if self.device >= 0:
            import torch

            s = torch.cuda.current_stream(self.device).cuda_stream
            self._check(self._lib.wlseno_set_stream(self._h, C.c_void_p(s)))

    def set_numeric_check(self, enable: bool = True):
        """Scan every later output for NaN/infinity; such an output raises
        WLSENOError with status ENUMERIC naming the first entry."""
        self._check(self._lib.wlseno_set_numeric_check(self._h, int(bool(enable))))

    # ------------------------------------------------------------ setup
    def mesh_upload(self, dim, verts, cells, periodic=False):
        v = np.ascontiguousarray(np.asarray(verts, dtype=np.float64).reshape(-1, dim))
        c = np.ascontiguousarray(np.asarray(cells, dtype=np.int32).reshape(-1, dim + 1))
        self._check(self._lib.wlseno_mesh_upload(
            self._h, int(dim), v.shape[0], v.ctypes.data_as(C.POINTER(C.c_double)), c.shape[0],
            c.ctypes.data_as(C.POINTER(C.c_int32)),
            (N.MESH_PERIODIC_1D if dim == 1 else N.MESH_PERIODIC_2D) if periodic else 0))
        self.dim = int(dim)
        self.n_cell = int(c.shape[0])

    def batch_add_mesh(self, dim, verts, cells) -> int:
        """Append one mesh to the context's batch; returns its index."""
        v = np.ascontiguousarray(np.asarray(verts, dtype=np.float64).reshape(-1, dim))
        c = np.ascontiguousarray(np.asarray(cells, dtype=np.int32).reshape(-1, dim + 1))
        mid = C.c_int32(-1)
        self._check(self._lib.wlseno_batch_add_mesh(
            self._h, int(dim), v.shape[0], v.ctypes.data_as(C.POINTER(C.c_double)), c.shape[0],
            c.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(mid)))
        self.dim = int(dim)
        self.n_cell = (self.n_cell or 0) + int(c.shape[0]) if mid.value > 0 else int(c.shape[0])
        return mid.value

    @staticmethod
    def _params(lib, p=3, n_lo=12, n_hi=20, flux="advection", velocity=(1.0, 0.0, 0.0), eps=1e-2, alpha_w=1.5,
                rank_tol=1e-12, weight_mode=0, gamma=1.4, lanes=0, bc=0, characteristic=False, far_state=None,
                balance=False, lf_alpha=0, h_mode=0):
        prm = N.Params()
        lib.wlseno_params_default(C.byref(prm))
        prm.p, prm.n_lo, prm.n_hi = int(p), int(n_lo), int(n_hi)
        prm.flux = N.FLUX[flux] if isinstance(flux, str) else int(flux)
        prm.weight_mode = int(weight_mode)
        prm.lanes = int(lanes)
        prm.bc = int(bc)
        prm.characteristic = int(bool(characteristic))
        prm.balance = int(bool(balance))
        prm.lf_alpha = int(lf_alpha)
        prm.h_mode = int(h_mode)
        for v in range(5):
            prm.far_state[v] = float(far_state[v]) if far_state is not None and v < len(far_state) else 0.0
        prm.eps, prm.alpha_w, prm.rank_tol, prm.gamma = float(eps), float(alpha_w), float(rank_tol), float(gamma)
        for d in range(3):
            prm.velocity[d] = float(velocity[d]) if d < len(velocity) else 0.0
        return prm

    def batch_params(self, dim, **kw):
        """Parameters (as stencil_build's keywords) for the batch's meshes of one dim; none: drop them."""
        prm = self._params(self._lib, **kw) if kw else None
        self._check(self._lib.wlseno_batch_params(self._h, int(dim), C.byref(prm) if prm is not None else None))

    def stencil_build(self, p=3, n_lo=12, n_hi=20, flux="advection", velocity=(1.0, 0.0, 0.0), eps=1e-2,
                      alpha_w=1.5, rank_tol=1e-12, weight_mode=0, gamma=1.4, lanes=0, bc=0, characteristic=False,
                      far_state=None, balance=False, lf_alpha=0, h_mode=0):
        prm = N.Params()
        self._lib.wlseno_params_default(C.byref(prm))
        prm.p, prm.n_lo, prm.n_hi = int(p), int(n_lo), int(n_hi)
        prm.flux = N.FLUX[flux] if isinstance(flux, str) else int(flux)
        prm.weight_mode = int(weight_mode)
        prm.lanes = int(lanes)
        prm.bc = int(bc)
        prm.characteristic = int(bool(characteristic))
        prm.balance = int(bool(balance))
        prm.lf_alpha = int(lf_alpha)
        prm.h_mode = int(h_mode)
        for v in range(5):
            prm.far_state[v] = float(far_state[v]) if far_state is not None and v < len(far_state) else 0.0
        prm.eps, prm.alpha_w, prm.rank_tol, prm.gamma = float(eps), float(alpha_w), float(rank_tol), float(gamma)
        for d in range(3):
            prm.velocity[d] = float(velocity[d]) if d < len(velocity) else 0.0
        self._check(self._lib.wlseno_stencil_build(self._h, C.byref(prm)))
        self.flux = flux
        self.characteristic = bool(characteristic)
        self._record_tag = None

    def info(self) -> dict:
        inf = N.Info()
        self._check(self._lib.wlseno_get_info(self._h, C.byref(inf)))
        return {k: getattr(inf, k) for k, _ in N.Info._fields_}

    def stencil(self):
        inf = self.info()
        rp = np.zeros(inf["n_cell"] + 1, dtype=np.int32)
        col = np.zeros(inf["nnz"], dtype=np.int32)
        self._check(self._lib.wlseno_get_stencil(self._h, rp.ctypes.data_as(C.POINTER(C.c_int32)),
                                                 col.ctypes.data_as(C.POINTER(C.c_int32))))
        return rp, col

    # ------------------------------------------------------------ device
    def _field(self, u):
        import torch

        if not (isinstance(u, torch.Tensor) and u.is_cuda and u.dtype == torch.float64 and u.is_contiguous()):
            raise TypeError("expected a contiguous float64 CUDA tensor")
        if u.numel() != self.info()["n_vars"] * self.n_cell:
            raise ValueError("field has the wrong number of entries")
        return u

    def reconstruct(self, u, coef=True, facevals=True, rank=True):
        import torch

        u = self._field(u)
        inf = self.info()
        V, nc = inf["n_vars"], inf["n_cell"]
        out = {}
        if coef and getattr(self, "characteristic", False):
            coef = False        # one fit per facet: no per-cell coefficients
        if coef:
            out["coef"] = torch.empty((V, nc, inf["m"]), dtype=torch.float64, device=u.device)
        if facevals:
            out["fval"] = torch.empty((V, nc, inf["faces_per_cell"], inf["points_per_face"]),
                                      dtype=torch.float64, device=u.device)
        if rank:
            out["rank"] = torch.empty((V, nc), dtype=torch.int32, device=u.device)
        self._sync_stream()
        self._check(self._lib.wlseno_reconstruct(self._h, _ptr(u), _ptr(out.get("coef")), _ptr(out.get("fval")),
                                                 _ptr(out.get("rank"))))
        return out

    def rhs(self, u, out=None):
        import torch

        u = self._field(u)
        if out is None:
            out = torch.empty_like(u)
        self._sync_stream()
        self._check(self._lib.wlseno_rhs(self._h, _ptr(u), _ptr(out)))
        return out

    def rhs_noalloc(self, u, out):
        """rhs() through the allocation-free entry point (scratch in the
        library's static per-GPU array); out must be preallocated."""
        u = self._field(u)
        out = self._field(out)
        self._sync_stream()
        self._check(self._lib.wlseno_rhs_noalloc(self._h, _ptr(u), _ptr(out)))
        return out

    def step(self, u, dt, n_steps):
        """Advance u in place by n_steps TVD RK3 steps of size dt."""
        u = self._field(u)
        self._sync_stream()
        self._check(self._lib.wlseno_step(self._h, _ptr(u), float(dt), int(n_steps)))
        return u

    def set_graphs(self, enable: bool):
        """Replay RK3 step pairs from a captured HIP graph (default) or launch directly."""
        self._check(self._lib.wlseno_set_graphs(self._h, 1 if enable else 0))

    def autotune(self, u=None) -> dict:
        """Time every compiled lane count of the reconstruction on this mesh
        (on u, or a synthetic smooth state) and keep the fastest."""
        t = N.Tune()
        if u is not None:
            u = self._field(u)
        self._sync_stream()
        self._check(self._lib.wlseno_autotune(self._h, _ptr(u) if u is not None else None, C.byref(t)))
        return {"chosen": t.chosen, "cached": bool(t.cached),
                "timings_us": {int(t.lanes[i]): float(t.us[i]) for i in range(t.n)}}

    STEP_MODES = {"direct": 0, "graphs": 1, "persistent": 2}

    def set_step_mode(self, mode):
        """'direct', 'graphs' (default) or 'persistent' (one cooperative launch for all steps)."""
        m = self.STEP_MODES[mode] if isinstance(mode, str) else int(mode)
        self._check(self._lib.wlseno_set_step_mode(self._h, m))

    def batch_step(self, u, dts, n_steps):
        """Advance a batch in place by n_steps TVD RK3 steps, mesh k with dts[k]."""
        u = self._field(u)
        d = np.ascontiguousarray(np.asarray(dts, dtype=np.float64))
        self._sync_stream()
        self._check(self._lib.wlseno_batch_step(self._h, _ptr(u), d.ctypes.data_as(C.POINTER(C.c_double)),
                                                int(n_steps)))
        return u

    def batch_last_alpha(self):
        a = np.zeros(self.info()["n_mesh"])
        self._sync_stream()
        self._check(self._lib.wlseno_batch_last_alpha(self._h, a.ctypes.data_as(C.POINTER(C.c_double))))
        return a

    # ----------------------------------------------------------- adjoint
    def rhs_vjp(self, u, v, out=None):
        """J(u)^T v for the advection right-hand side L."""
        import torch

        u = self._field(u)
        v = self._field(v)
        if out is None:
            out = torch.empty_like(u)
        self._sync_stream()
        self._check(self._lib.wlseno_rhs_vjp(self._h, _ptr(u), _ptr(v), _ptr(out)))
        return out

    def step_adjoint(self, u0, dt, n_steps, gT, ckpt_every=10, out=None):
        """(d u(T)/d u0)^T gT for n_steps TVD RK3 steps of size dt from u0."""
        import torch

        u0 = self._field(u0)
        gT = self._field(gT)
        if out is None:
            out = torch.empty_like(u0)
        self._sync_stream()
        self._check(self._lib.wlseno_step_adjoint(self._h, _ptr(u0), float(dt), int(n_steps), int(ckpt_every),
                                                  _ptr(gT), _ptr(out)))
        self._record_tag = None      # the library dropped any recorded trajectory
        return out

    def step_record(self, u, dt, n_steps, ckpt_every=10):
        """step() that keeps checkpoints for step_adjoint_recorded()."""
        u = self._field(u)
        self._sync_stream()
        self._check(self._lib.wlseno_step_record(self._h, _ptr(u), float(dt), int(n_steps), int(ckpt_every)))
        return u

    def step_adjoint_recorded(self, gT, out=None):
        """(d u(T)/d u0)^T gT for the trajectory of the last step_record()."""
        import torch

        gT = self._field(gT)
        if out is None:
            out = torch.empty_like(gT)
        self._sync_stream()
        self._check(self._lib.wlseno_step_adjoint_recorded(self._h, _ptr(gT), _ptr(out)))
        return out

    def last_alpha(self) -> float:
        a = C.c_double(0.0)
        self._sync_stream()
        self._check(self._lib.wlseno_last_alpha(self._h, C.byref(a)))
        return a.value

    # ---------------------------------------------------------- timing
    def time_kernel(self, kernel: int, u, launches: int) -> float:
        """Average milliseconds per launch of kernel 0 (reconstruction) or 1
        (flux/update) over `launches` back-to-back launches on state u."""
        u = self._field(u)
        ms = C.c_double(0.0)
        self._sync_stream()
        self._check(self._lib.wlseno_time_kernel(self._h, int(kernel), _ptr(u), int(launches), C.byref(ms)))
        return ms.value
