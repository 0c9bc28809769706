"""FP64 CPU oracle for the spectral TV decomposition (arXiv 2006.10004).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP library and never imports it.

The arithmetic lives in ``tvspec_oracle.c`` (plain C, double precision); this
module only marshals numpy arrays through ctypes.  Function-by-function
citations of the paper are in the C source:

  grad / div      discrete isotropic TV in dual form, Sec. 2.1 Eq. (2)
  rof             implicit Euler step of Eq. (1) = ROF problem Eq. (8),
                  Chambolle's dual fixed point (the solver named in Sec. 4.3)
  rof_pdhg        the same ROF problem by the Chambolle-Pock primal-dual
                  algorithm (the paper's GPU baseline solver, Sec. 4.3)
  tv_flow         the flow u_0 = f, u_{s+1} = ROF(u_s, dt)
  spectral        phi = t u_tt Eq. (3), S(t) = ||phi||_1, bands Eq. (7),
                  residual Eq. (5)
  decompose       tv_flow followed by spectral, per channel, with either
                  ROF solver

Parity status: every function is pinned by tests/test_oracle_*.py against
closed forms, invariants and brute force.  The finite-iteration path of both
ROF solvers is pinned by worked examples: the first iterates on a two-level
2 x 2 image, derived by hand as exact fractions.  A finite-iteration iterate
on a general image has no closed form.  There the pins are those examples,
the converged special cases and the invariants.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle_tvspec.so")
_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_fp = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")

DEFAULT_TAU = 0.248
# primal-dual steps tau = sigma = 1/sqrt(8): tau sigma ||grad||^2 <= 1
PDHG_STEP = 1.0 / np.sqrt(8.0)
SOLVERS = {"chambolle": 0, "pdhg": 1}


def _load():
    global _lib
    if _lib is not None:
        return _lib
    sanitized = os.environ.get("TVSPEC_ORACLE_SANITIZE") == "1"
    path = os.path.join(_HERE, "liboracle_tvspec_san.so") if sanitized else _LIB_PATH
    if not os.path.exists(path):
        from . import build as _b
        _b.build(sanitize=sanitized)
    lib = ctypes.CDLL(path)
    i, d = ctypes.c_int, ctypes.c_double
    lib.orc_num_threads.argtypes = []
    lib.orc_num_threads.restype = i
    lib.orc_grad.argtypes = [_dp, i, i, _dp, _dp]
    lib.orc_grad.restype = None
    lib.orc_div.argtypes = [_dp, _dp, i, i, _dp]
    lib.orc_div.restype = None
    lib.orc_tv.argtypes = [_dp, i, i]
    lib.orc_tv.restype = d
    lib.orc_rof.argtypes = [_dp, i, i, d, d, i, _dp, _dp, _dp]
    lib.orc_rof.restype = None
    lib.orc_tv_flow.argtypes = [_dp, i, i, d, i, i, d, i, _dp]
    lib.orc_tv_flow.restype = None
    lib.orc_spectral.argtypes = [_dp, i, i, d, i, _ip, i, _dp, _dp, _dp, ctypes.c_void_p]
    lib.orc_spectral.restype = None
    lib.orc_edges_valid.argtypes = [i, _ip, i]
    lib.orc_edges_valid.restype = i
    lib.orc_decompose.argtypes = [_fp, i, i, i, d, i, i, d, i, _ip, i, _dp, _dp, _dp, _dp]
    lib.orc_decompose.restype = i
    lib.orc_rof_pdhg.argtypes = [_dp, i, i, d, d, d, i, _dp, _dp, _dp]
    lib.orc_rof_pdhg.restype = None
    lib.orc_decompose_solver.argtypes = [_fp, i, i, i, d, i, i, i, d, d, i, _ip, i, _dp, _dp, _dp, _dp]
    lib.orc_decompose_solver.restype = i
    _lib = lib
    return lib


def num_threads():
    """Threads the oracle's per-pixel loops run on."""
    return int(_load().orc_num_threads())


def _plane(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim != 2 or a.shape[0] < 2 or a.shape[1] < 2:
        raise ValueError("expected an H x W array with H, W >= 2")
    return a


def grad(u):
    """Forward-difference gradient with Neumann boundary -> (gx, gy)."""
    u = _plane(u)
    H, W = u.shape
    gx = np.empty_like(u)
    gy = np.empty_like(u)
    _load().orc_grad(u, H, W, gx, gy)
    return gx, gy


def div(px, py):
    """Discrete divergence, the negative adjoint of grad."""
    px = _plane(px)
    py = _plane(py)
    H, W = px.shape
    d = np.empty_like(px)
    _load().orc_div(px, py, H, W, d)
    return d


def tv(u):
    """Discrete isotropic total variation sum |grad u|."""
    u = _plane(u)
    return _load().orc_tv(u, u.shape[0], u.shape[1])


def rof(g, lam, iters, tau=DEFAULT_TAU, px=None, py=None):
    """Chambolle's fixed point for min 0.5||g-v||^2 + lam TV(v).

    Returns (v, px, py); (px, py) start at zero unless given."""
    g = _plane(g)
    H, W = g.shape
    px = np.zeros_like(g) if px is None else np.array(px, dtype=np.float64, order="C")
    py = np.zeros_like(g) if py is None else np.array(py, dtype=np.float64, order="C")
    v = np.empty_like(g)
    _load().orc_rof(g, H, W, float(lam), float(tau), int(iters), px, py, v)
    return v, px, py


def rof_pdhg(g, lam, iters, tau=PDHG_STEP, sigma=PDHG_STEP, yx=None, yy=None):
    """Chambolle-Pock primal-dual iteration for min 0.5||g-v||^2 + lam TV(v),
    from x = xbar = g.  Returns (v, yx, yy); (yx, yy) start at zero unless
    given."""
    g = _plane(g)
    H, W = g.shape
    yx = np.zeros_like(g) if yx is None else np.array(yx, dtype=np.float64, order="C")
    yy = np.zeros_like(g) if yy is None else np.array(yy, dtype=np.float64, order="C")
    v = np.empty_like(g)
    _load().orc_rof_pdhg(g, H, W, float(lam), float(tau), float(sigma), int(iters), yx, yy, v)
    return v, yx, yy


def tv_flow(f, dt, nsteps, iters, tau=DEFAULT_TAU, warm=False):
    """States u_0..u_nsteps of the implicit-Euler TV flow, shape (nsteps+1, H, W).

    warm=False (default): every ROF solve starts its dual field at zero."""
    f = _plane(f)
    H, W = f.shape
    states = np.empty((nsteps + 1, H, W), dtype=np.float64)
    _load().orc_tv_flow(f, H, W, float(dt), int(nsteps), int(iters), float(tau),
                        1 if warm else 0, states)
    return states


def spectral(states, dt, K, edges, want_phi=False):
    """phi, S, bands and residual from stored states u_0..u_{K+1}.

    Returns dict(S (K,), bands (B,H,W), residual (H,W), phi (K,H,W) or None)."""
    states = np.ascontiguousarray(states, dtype=np.float64)
    if states.shape[0] < K + 2:
        raise ValueError("need states u_0..u_{K+1}")
    H, W = states.shape[1:]
    e = np.ascontiguousarray(edges, dtype=np.int32)
    B = len(e) - 1
    if not _load().orc_edges_valid(int(K), e, B):
        raise ValueError("invalid band edges")
    S = np.empty(K)
    bands = np.empty((B, H, W))
    res = np.empty((H, W))
    phi = np.empty((K, H, W)) if want_phi else None
    _load().orc_spectral(states, H, W, float(dt), int(K), e, B, S, bands, res,
                         phi.ctypes.data if want_phi else None)
    return {"S": S, "bands": bands, "residual": res, "phi": phi}


def decompose(f, dt, K, iters, edges, tau=None, warm=False, solver="chambolle", sigma=None):
    """Full decomposition of a (C,H,W) or (H,W) float32 image.

    warm=False (default): every ROF solve starts its dual field at zero (the
    paper does not say how the dual field is initialised; see tv_flow).
    solver "chambolle" (step tau, default 0.248) or "pdhg" (steps tau and
    sigma, default 1/sqrt(8) each).

    Returns dict(bands (B,C,H,W), S (C,K), residual (C,H,W), recon_err, mean_err)."""
    f = np.asarray(f)
    if f.ndim == 2:
        f = f[None]
    f = np.ascontiguousarray(f, dtype=np.float32)
    C, H, W = f.shape
    e = np.ascontiguousarray(edges, dtype=np.int32)
    B = len(e) - 1
    bands = np.empty((B, C, H, W))
    S = np.empty((C, K))
    res = np.empty((C, H, W))
    rep = np.empty(2)
    sv = SOLVERS[solver]
    if tau is None:
        tau = PDHG_STEP if sv == 1 else DEFAULT_TAU
    if sigma is None:
        sigma = PDHG_STEP if sv == 1 else 0.0
    rc = _load().orc_decompose_solver(f, H, W, C, float(dt), int(K), int(iters), sv, float(tau), float(sigma),
                                      1 if warm else 0, e, B, bands, S, res, rep)
    if rc != 0:
        raise ValueError("invalid arguments to the oracle decomposition")
    return {"bands": bands, "S": S, "residual": res,
            "recon_err": float(rep[0]), "mean_err": float(rep[1])}


def dyadic_edges(K, nbands):
    """Dyadic step-index edges {0, 1, 2, 4, ..., 2^(B-2), K} (the paper's
    dyadic grouping of unit-step bands, Sec. 4.1)."""
    if nbands < 1:
        raise ValueError("nbands >= 1")
    if nbands == 1:
        return [0, K]
    e = [0] + [2 ** j for j in range(nbands - 1)] + [K]
    if e[-2] >= K:
        raise ValueError("2^(B-2) must be < K")
    return e
