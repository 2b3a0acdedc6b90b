"""ctypes harness around the oracle's C numerical core.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

from .mesh import OracleMesh

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wlseno_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_LIB_LD = os.path.join(_HERE, "liboracle_ld.so")
_LIB_TAN = os.path.join(_HERE, "liboracle_tan.so")
_TAN_HDR = os.path.join(_HERE, "tangent.hpp")

FLUX = {"advection": 0, "burgers": 1, "euler": 2}


def build(force: bool = False, extended: bool = False, tangent: bool = False) -> str:
    """Compile the C core with gcc (-O2 -ffp-contract=off, OpenMP).  The
    extended build runs the same algorithm in x87 long double; it is used only
    to measure the FP64 rounding floor of individual cells.  The tangent build
    compiles the same file as C++ on the dual numbers of tangent.hpp (values
    bitwise those of the FP64 build, plus exact directional derivatives on
    the active branch); stencils up to 64 rows and 15 coefficients."""
    out = _LIB_TAN if tangent else (_LIB_LD if extended else _LIB)
    deps = [_SRC] + ([_TAN_HDR] if tangent else [])
    if force or not os.path.exists(out) or any(os.path.getmtime(out) < os.path.getmtime(d) for d in deps):
        tmp = out + ".tmp"
        if tangent:
            cmd = ["g++", "-x", "c++", "-std=c++17", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                   "-include", _TAN_HDR, "-DOR_REAL=or_dual", "-DOR_GREAL=double", "-DOR_TANGENT", "-DOR_MAXM=15", "-DOR_MAXN=64"]
        else:
            cmd = ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c99"]
            if extended:
                cmd.append("-DOR_REAL=long double")
        cmd += ["-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, out)
    return out


_libs = {}


def lib(extended: bool = False, tangent: bool = False):
    key = "tan" if tangent else ("ld" if extended else "fp64")
    _lib = _libs.get(key)
    if _lib is None:
        _lib = C.CDLL(build(extended=extended, tangent=tangent))
        _libs[key] = _lib
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        _lib.or_num_coeffs.argtypes = [C.c_int, C.c_int]
        _lib.or_basis.argtypes = [C.c_int, C.c_int, ip]
        _lib.or_simplex_avg_monomial.argtypes = [C.c_int, dp, dp, ip]
        _lib.or_simplex_avg_monomial.restype = C.c_double
        _lib.or_wls_qrcp_solve.argtypes = [C.c_int, C.c_int, dp, dp, dp, C.c_double, dp, dp, ip]
        _lib.or_eval_taylor.argtypes = [C.c_int, C.c_int, ip, dp, dp]
        _lib.or_eval_taylor.restype = C.c_double
        _lib.or_char_basis.argtypes = [C.c_int, C.c_double, dp, dp, dp, dp]
        _lib.or_euler_normal_flux.argtypes = [C.c_int, C.c_double, dp, dp, dp]
        pp = C.POINTER(_Problem)
        _lib.or_balanced_rows.argtypes = [pp, C.c_int, dp, C.c_int, ip]
        _lib.or_cell_matrix.argtypes = [pp, C.c_int, dp]
        _lib.or_cell_weights.argtypes = [pp, C.c_int, dp, dp]
        ub = C.POINTER(C.c_ubyte)
        _lib.or_reconstruct.argtypes = [pp, dp, dp, dp, ip, ub, ub]
        _lib.or_reconstruct_cells.argtypes = [pp, dp, C.c_int, ip, dp, dp, ip, ub, ub]
        _lib.or_rhs.argtypes = [pp, dp, dp, dp]
        _lib.or_rk3.argtypes = [pp, dp, C.c_double, C.c_int]
        _lib.or_num_threads.argtypes = []
        _lib.or_set_num_threads.argtypes = [C.c_int]
        if tangent:
            _lib.or_ndir.argtypes = []
            _lib.or_rhs_tangent.argtypes = [pp, dp, dp, C.c_int, dp, dp]
            _lib.or_rk3_tangent.argtypes = [pp, dp, dp, C.c_int, C.c_double, C.c_int]
    return _lib


def num_threads() -> int:
    return int(lib().or_num_threads())


def set_num_threads(n: int) -> int:
    """Threads of the FP64 build's per-cell loops from now on; returns the previous count."""
    return int(lib().or_set_num_threads(int(n)))


class _Problem(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("p", C.c_int), ("m", C.c_int), ("nvars", C.c_int),
        ("flux", C.c_int), ("weight_mode", C.c_int),
        ("nc", C.c_int), ("nq", C.c_int), ("periodic", C.c_int), ("bc", C.c_int), ("characteristic", C.c_int),
        ("period", C.c_double), ("eps", C.c_double), ("alpha_w", C.c_double),
        ("rank_tol", C.c_double), ("h", C.c_double), ("gamma", C.c_double),
        ("adv", C.c_double * 3),
        ("far", C.c_double * 5),
        ("exps", C.POINTER(C.c_int)),
        ("cv", C.POINTER(C.c_double)),
        ("cent", C.POINTER(C.c_double)),
        ("vol", C.POINTER(C.c_double)),
        ("nbr", C.POINTER(C.c_int)),
        ("row_ptr", C.POINTER(C.c_int)),
        ("col", C.POINTER(C.c_int)),
        ("qx", C.POINTER(C.c_double)),
        ("qw", C.POINTER(C.c_double)),
        ("normal", C.POINTER(C.c_double)),
        ("area", C.POINTER(C.c_double)),
        ("pool_ptr", C.POINTER(C.c_int)),
        ("pool_col", C.POINTER(C.c_int)),
        ("balance", C.c_int),
        ("period_y", C.c_double),
        ("lf_alpha", C.c_int),
        ("h_cell", C.POINTER(C.c_double)),
    ]


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def num_coeffs(dim: int, p: int) -> int:
    return int(lib().or_num_coeffs(dim, p))


def basis(dim: int, p: int) -> np.ndarray:
    m = num_coeffs(dim, p)
    exps = np.zeros((m, 3), dtype=np.int32)
    lib().or_basis(dim, p, _ip(exps))
    return exps


def simplex_avg_monomial(verts, center, a) -> float:
    verts = np.ascontiguousarray(verts, dtype=np.float64)
    dim = verts.shape[1]
    c = np.ascontiguousarray(center, dtype=np.float64)
    a = np.ascontiguousarray(list(a) + [0] * (3 - len(a)), dtype=np.int32)
    return float(lib().or_simplex_avg_monomial(dim, _dp(verts), _dp(c), _ip(a)))


def char_basis(dim, gamma, U, n):
    """(L, R) of the Euler normal-flux Jacobian at state U along unit normal n."""
    V = dim + 2
    U = np.ascontiguousarray(U, dtype=np.float64)
    n = np.ascontiguousarray(n, dtype=np.float64)
    L = np.zeros((V, V))
    R = np.zeros((V, V))
    if lib().or_char_basis(int(dim), float(gamma), _dp(U), _dp(n), _dp(L), _dp(R)):
        raise ValueError("characteristic basis: 1-D and 2-D only")
    return L, R


def euler_normal_flux(dim, gamma, U, n):
    U = np.ascontiguousarray(U, dtype=np.float64)
    n = np.ascontiguousarray(n, dtype=np.float64)
    F = np.zeros(dim + 2)
    lib().or_euler_normal_flux(int(dim), float(gamma), _dp(U), _dp(n), _dp(F))
    return F


def wls_qrcp_solve(A, w, b, rank_tol: float = 1e-12):
    """Column-scaled weighted LS by Householder QRCP; returns (v, rank, rdiag, perm)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    n, m = A.shape
    w = np.ascontiguousarray(w, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    v = np.zeros(m)
    rd = np.zeros(min(n, m))
    perm = np.zeros(m, dtype=np.int32)
    r = lib().or_wls_qrcp_solve(n, m, _dp(A), _dp(w), _dp(b), rank_tol, _dp(v), _dp(rd), _ip(perm))
    return v, int(r), rd, perm


def eval_taylor(dim, exps, v, dx) -> float:
    exps = np.ascontiguousarray(exps, dtype=np.int32)
    v = np.ascontiguousarray(v, dtype=np.float64)
    dx = np.ascontiguousarray(list(dx) + [0.0] * (3 - len(dx)), dtype=np.float64)
    return float(lib().or_eval_taylor(dim, exps.shape[0], _ip(exps), _dp(v), _dp(dx)))


class Oracle:
    """FP64 reference of the WLS-ENO finite-volume right-hand side and RK3 step."""

    def __init__(self, dim, verts, cells, periodic=False, *, p=3, n_lo=None, n_hi=None,
                 flux="advection", velocity=(1.0, 0.0, 0.0), eps=1e-2, alpha_w=1.5,
                 rank_tol=1e-12, gamma=1.4, weight_mode=0, stencil=None, h=None, extended=False, bc=0,
                 characteristic=False, far_state=None, balance=False, lf_alpha=0, h_mode=0, tangent=False):
        self.extended = bool(extended)
        self.tangent = bool(tangent)
        if self.tangent and self.extended:
            raise ValueError("the tangent build is FP64")
        self.mesh = OracleMesh(dim, verts, cells, periodic, p=p)
        om = self.mesh
        self.dim, self.p, self.nc = om.dim, int(p), om.nc
        self.exps = basis(dim, p)
        self.m = self.exps.shape[0]
        self.nvars = dim + 2 if flux == "euler" else 1
        if n_lo is None:
            n_lo = self.m
        if n_hi is None:
            n_hi = 2 * self.m
        self.n_lo, self.n_hi = int(n_lo), int(n_hi)
        if stencil is None:
            stencil = om.stencils(self.n_lo, self.n_hi)
        self.row_ptr = np.ascontiguousarray(stencil[0], dtype=np.int32)
        self.col = np.ascontiguousarray(stencil[1], dtype=np.int32)
        self.h = om.h if h is None else float(h)
        self._keep = dict(
            exps=np.ascontiguousarray(self.exps, dtype=np.int32),
            cv=np.ascontiguousarray(om.cv, dtype=np.float64),
            cent=np.ascontiguousarray(om.cent, dtype=np.float64),
            vol=np.ascontiguousarray(om.vol, dtype=np.float64),
            nbr=np.ascontiguousarray(om.nbr, dtype=np.int32),
            qx=np.ascontiguousarray(om.qx, dtype=np.float64),
            qw=np.ascontiguousarray(om.qw, dtype=np.float64),
            normal=np.ascontiguousarray(om.normal, dtype=np.float64),
            area=np.ascontiguousarray(om.area, dtype=np.float64),
        )
        k = self._keep
        P = _Problem()
        P.dim, P.p, P.m, P.nvars = om.dim, self.p, self.m, self.nvars
        P.flux, P.weight_mode = FLUX[flux], int(weight_mode)
        P.nc, P.nq, P.periodic = om.nc, om.nq, int(om.periodic)
        P.bc = int(bc)
        if characteristic and (flux != "euler" or dim > 2):
            raise ValueError("characteristic fields: the 1-D and 2-D Euler system only")
        P.characteristic = int(bool(characteristic))
        if bc == 3 and flux != "euler":
            raise ValueError("bc = 3 (slip wall): the Euler system only")
        for v in range(5):
            P.far[v] = float(far_state[v]) if far_state is not None and v < len(far_state) else 0.0
        P.period, P.eps, P.alpha_w, P.rank_tol = om.period, eps, alpha_w, rank_tol
        P.period_y = om.period_y
        P.h, P.gamma = self.h, gamma
        for d in range(3):
            P.adv[d] = float(velocity[d]) if d < len(velocity) else 0.0
        P.exps = _ip(k["exps"])
        P.cv, P.cent, P.vol = _dp(k["cv"]), _dp(k["cent"]), _dp(k["vol"])
        P.nbr = _ip(k["nbr"])
        P.row_ptr, P.col = _ip(self.row_ptr), _ip(self.col)
        P.qx, P.qw = _dp(k["qx"]), _dp(k["qw"])
        P.normal, P.area = _dp(k["normal"]), _dp(k["area"])
        if balance:
            if flux == "euler":
                raise ValueError("balanced stencils: scalar fluxes only")
            # enlarged stencils: the same rule with twice the sizes
            pool = om.stencils(2 * self.n_lo, 2 * self.n_hi)
            self.pool_ptr = np.ascontiguousarray(pool[0], dtype=np.int32)
            self.pool_col = np.ascontiguousarray(pool[1], dtype=np.int32)
            P.pool_ptr, P.pool_col = _ip(self.pool_ptr), _ip(self.pool_col)
        P.balance = int(bool(balance))
        P.lf_alpha = int(lf_alpha)
        if h_mode:
            # h_i: the mean length of cell i's edges (1-D: its width)
            self.h_cell = np.ascontiguousarray(om.cell_mean_edge(), dtype=np.float64)
            P.h_cell = _dp(self.h_cell)
        self._P = P
        self._lib = lib(self.extended, self.tangent)
        if self.tangent and (self.m > 15 or int(np.max(np.diff(self.row_ptr))) > 64):
            raise ValueError("the tangent build holds stencils up to 64 rows and 15 coefficients")
        self.flux = flux
        self.nq = om.nq
        self.nf = dim + 1

    # -------------------------------------------------------------- pieces
    def balanced_rows(self, i, grad, n):
        """Balanced stencil of cell i for gradient grad and size n (needs balance=True)."""
        out = np.zeros(2 * self.n_hi + 1, dtype=np.int32)
        g = np.ascontiguousarray(grad, dtype=np.float64)
        k = self._lib.or_balanced_rows(C.byref(self._P), int(i), _dp(g), int(n), _ip(out))
        return out[:k].copy()

    def stencil_of(self, i):
        return self.col[self.row_ptr[i]:self.row_ptr[i + 1]]

    def cell_matrix(self, i):
        n = int(self.row_ptr[i + 1] - self.row_ptr[i])
        A = np.zeros((n, self.m))
        self._lib.or_cell_matrix(C.byref(self._P), int(i), _dp(A))
        return A

    def cell_weights(self, i, u):
        u = np.ascontiguousarray(u, dtype=np.float64)
        n = int(self.row_ptr[i + 1] - self.row_ptr[i])
        w = np.zeros(n)
        self._lib.or_cell_weights(C.byref(self._P), int(i), _dp(u), _dp(w))
        return w

    def _u(self, u):
        u = np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape(self.nvars, self.nc))
        return u

    def reconstruct(self, u, cells=None):
        """Coefficients (V, nc, m), facet values (V, nc, F, Q), ranks (V, nc), fallback (nc)."""
        u = self._u(u)
        coef = np.zeros((self.nvars, self.nc, self.m))
        fval = np.zeros((self.nvars, self.nc, self.nf, self.nq))
        rank = np.zeros((self.nvars, self.nc), dtype=np.int32)
        fb = np.zeros(self.nc, dtype=np.uint8)
        rb = np.zeros(self.nc, dtype=np.uint8)
        fbp = fb.ctypes.data_as(C.POINTER(C.c_ubyte))
        rbp = rb.ctypes.data_as(C.POINTER(C.c_ubyte))
        if cells is None:
            self._lib.or_reconstruct(C.byref(self._P), _dp(u), _dp(coef), _dp(fval), _ip(rank), fbp, rbp)
        else:
            cells = np.ascontiguousarray(cells, dtype=np.int32)
            self._lib.or_reconstruct_cells(C.byref(self._P), _dp(u), len(cells), _ip(cells),
                                       _dp(coef), _dp(fval), _ip(rank), fbp, rbp)
        return dict(coef=coef, fval=fval, rank=rank, fallback=fb, rebalanced=rb)

    def rhs(self, u):
        u = self._u(u)
        out = np.zeros_like(u)
        alpha = C.c_double(0.0)
        if self._lib.or_rhs(C.byref(self._P), _dp(u), _dp(out), C.byref(alpha)):
            raise MemoryError("oracle rhs allocation failed")
        return out, alpha.value

    def step(self, u, dt, nsteps):
        u = self._u(u).copy()
        if self._lib.or_rk3(C.byref(self._P), _dp(u), float(dt), int(nsteps)):
            raise MemoryError("oracle rk3 allocation failed")
        return u

    # ----------------------------------------------------------- tangents
    def _dirs(self, dirs):
        d = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64).reshape(-1, self.nvars * self.nc))
        return d

    def rhs_tangent(self, u, dirs):
        """L(u) and J(u) d for every direction d (rows of dirs), exact on the
        active branch (tangent build only)."""
        if not self.tangent:
            raise ValueError("construct the oracle with tangent=True")
        u = self._u(u)
        D = self._dirs(dirs)
        width = int(self._lib.or_ndir())
        L = np.zeros_like(u)
        JD = np.zeros_like(D)
        for k0 in range(0, max(D.shape[0], 1), width):
            blk = np.ascontiguousarray(D[k0:k0 + width])
            out = np.zeros_like(blk)
            if self._lib.or_rhs_tangent(C.byref(self._P), _dp(u), _dp(blk), blk.shape[0], _dp(L), _dp(out)):
                raise MemoryError("oracle tangent rhs failed")
            JD[k0:k0 + width] = out
        return L, JD

    def step_tangent(self, u, dirs, dt, nsteps):
        """u(T) after nsteps RK3 steps and (d u(T) / d u0) d for every
        direction d (rows of dirs): the exact tangent of the trajectory on its
        active branch (tangent build only).  Directions run or_ndir() at a time."""
        if not self.tangent:
            raise ValueError("construct the oracle with tangent=True")
        u0 = self._u(u)
        D = self._dirs(dirs)
        width = int(self._lib.or_ndir())
        uT = None
        JD = np.zeros_like(D)
        for k0 in range(0, max(D.shape[0], 1), width):
            us = u0.copy()
            blk = np.ascontiguousarray(D[k0:k0 + width]).copy()
            if self._lib.or_rk3_tangent(C.byref(self._P), _dp(us), _dp(blk), blk.shape[0], float(dt), int(nsteps)):
                raise MemoryError("oracle tangent rk3 failed")
            JD[k0:k0 + width] = blk
            uT = us
        return uT, JD


def from_workload(wl, **kw) -> Oracle:
    s = dict(wl.settings)
    args = dict(p=s["p"], n_lo=s["n_lo"], n_hi=s["n_hi"], flux=s["flux"],
                velocity=s.get("velocity", (1.0, 0.0, 0.0)), gamma=s.get("gamma", 1.4), bc=s.get("bc", 0),
                characteristic=s.get("characteristic", False), far_state=s.get("far_state"),
                balance=s.get("balance", False))
    args.update(kw)
    return Oracle(wl.mesh.dim, wl.mesh.verts, wl.mesh.cells, wl.mesh.periodic, **args)
