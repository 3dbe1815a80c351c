"""FP64 oracle for parallel-in-sequence MCMC -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP library
in ``paper_2508_18413_amd``; the two meet only at the seeded input arrays.

Contents
--------
* ctypes bindings of ``oracle.c`` (targets, sequential MALA/ULA/HMC chains,
  whole HMC transitions as chain steps with their Jacobians, step Jacobians,
  sequential linear recursions, tangent/adjoint derivatives);
* ``newton_reference``: Algorithm 1 of the paper (Appendix A.1) in FP64, the
  linearised recursion of Sec. 2 eq. 2/3 (dense), eq. 4 (diagonal), the block
  quasi-DEER recursion of Appendix A.3, Picard (J = 0), or the diagonal
  estimated from one Rademacher probe per step and sweep (Sec. 3.4 eq. 10),
  solved by a plain sequential loop;
* ``probe_sign`` / ``splitmix64``: the counter-based signs of that probe;
* ``damp_and_clip``: the damped, entrywise- or norm-clipped Jacobian of full
  DEER;
* ``rotated_provider``: the chain in orthogonally rotated coordinates
  (Sec. 3.4 eq. 11), whose quasi-DEER diagonal is diag(Q^T J Q);
* ``bidiagonal_bruteforce``: the Newton linear system written as one block
  lower-bidiagonal matrix and solved by LAPACK (numpy.linalg.solve).

Parity pins of every function live in ``tests/test_oracle_*.py``.  Functions
documented there as "parity unpinned" have no pin beyond oracle agreement.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")

GAUSSIAN, BANANA, LOGREG, FUNNEL = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc into liboracle.so (plain -O2, no fast-math)."""
    if force or not os.path.exists(_SO):
        src = os.path.join(_HERE, "oracle.c")
        tmp = _SO + ".tmp"
        subprocess.run(["gcc", "-O2", "-fno-fast-math", "-fno-tree-vectorize", "-std=c11",
                        "-fPIC", "-shared", "-o", tmp, src, "-lm"], check=True)
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = C.CDLL(_SO)
        dp = C.POINTER(C.c_double)
        bp = C.POINTER(C.c_int8)
        L.orc_logp.restype = C.c_double
        L.orc_logp.argtypes = [C.c_void_p, dp]
        L.orc_grad.argtypes = [C.c_void_p, dp, dp]
        L.orc_hess.argtypes = [C.c_void_p, dp, dp]
        L.orc_dgrad_dtheta.argtypes = [C.c_void_p, dp, dp]
        L.orc_dlogp_dtheta.restype = C.c_double
        L.orc_dlogp_dtheta.argtypes = [C.c_void_p, dp]
        L.orc_mala_step.restype = C.c_int
        L.orc_mala_step.argtypes = [C.c_void_p, C.c_double, C.c_int, dp, dp, C.c_double, C.c_int,
                                    dp, dp, dp, dp]
        L.orc_mala_chain.restype = C.c_long
        L.orc_mala_chain.argtypes = [C.c_void_p, C.c_double, C.c_int, C.c_long, dp, dp, dp, bp,
                                     dp, bp, dp]
        L.orc_mala_jac.restype = C.c_int
        L.orc_mala_jac.argtypes = [C.c_void_p, C.c_double, C.c_int, C.c_int, dp, dp, C.c_double,
                                   C.c_int, dp, dp]
        L.orc_mala_smoothed_step.argtypes = [C.c_void_p, C.c_double, dp, dp, C.c_double, dp]
        L.orc_leapfrog_step.argtypes = [C.c_void_p, C.c_double, dp, dp, dp]
        L.orc_hmc_chain.restype = C.c_long
        L.orc_hmc_chain.argtypes = [C.c_void_p, C.c_double, C.c_int, C.c_long, dp, dp, dp, bp,
                                    dp, bp, dp, dp, dp]
        L.orc_hmc_step.restype = C.c_int
        L.orc_hmc_step.argtypes = [C.c_void_p, C.c_double, C.c_int, dp, dp, dp, C.c_double, C.c_int,
                                   dp, dp, dp, dp]
        L.orc_hmc_seq_chain.restype = C.c_long
        L.orc_hmc_seq_chain.argtypes = [C.c_void_p, C.c_double, C.c_int, dp, C.c_long, dp, dp, dp, bp,
                                        dp, bp, dp]
        L.orc_hmc_step_jac.restype = C.c_int
        L.orc_hmc_step_jac.argtypes = [C.c_void_p, C.c_double, C.c_int, dp, C.c_int, dp, dp, C.c_double,
                                       C.c_int, dp, dp]
        L.orc_hmc_smoothed_step.argtypes = [C.c_void_p, C.c_double, C.c_int, dp, dp, dp, C.c_double, dp]
        L.orc_linrec_diag.argtypes = [C.c_long, C.c_int, dp, dp, dp]
        L.orc_linrec_dense.argtypes = [C.c_long, C.c_int, dp, dp, dp]
        L.orc_linrec_block2.argtypes = [C.c_long, C.c_int, dp, dp, dp, dp, dp, dp, dp, dp]
        L.orc_mala_tangent.argtypes = [C.c_void_p, C.c_double, C.c_int, C.c_long, dp, dp, dp, bp,
                                       dp, dp]
        L.orc_mala_adjoint.argtypes = [C.c_void_p, C.c_double, C.c_int, C.c_long, dp, dp, dp, bp,
                                       dp, dp, dp]
        _lib = L
    return _lib


def _d(a):
    """FP64 C-contiguous view/copy and its data pointer."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def _nullable(a, kind):
    if a is None:
        return None, None
    a = np.ascontiguousarray(a, dtype=np.float64 if kind == "d" else np.int8)
    ptr = a.ctypes.data_as(C.POINTER(C.c_double if kind == "d" else C.c_int8))
    return a, ptr


class _TargetStruct(C.Structure):
    _fields_ = [("kind", C.c_int), ("dim", C.c_int), ("mean", C.c_void_p), ("prec", C.c_void_p),
                ("X", C.c_void_p), ("y", C.c_void_p), ("n", C.c_int), ("prior_var", C.c_double),
                ("theta", C.c_double)]


class Target:
    """A target density for the oracle.  Arrays are promoted exactly to FP64."""

    MAX_DIM = 1024  # capacity of oracle.c's per-call arrays

    def __init__(self, kind, dim, mean=None, prec=None, X=None, y=None, prior_var=1.0, theta=0.0):
        self.kind, self.dim = int(kind), int(dim)
        if not 1 <= self.dim <= self.MAX_DIM:
            raise ValueError(f"oracle targets have 1 <= dim <= {self.MAX_DIM} (got {self.dim})")
        self._keep = []
        s = _TargetStruct()
        s.kind, s.dim, s.prior_var, s.theta = self.kind, self.dim, float(prior_var), float(theta)
        if mean is not None:
            m = np.ascontiguousarray(mean, dtype=np.float64)
            self._keep.append(m)
            s.mean = m.ctypes.data
        if prec is not None:
            p = np.ascontiguousarray(prec, dtype=np.float64)
            self._keep.append(p)
            s.prec = p.ctypes.data
        if X is not None:
            x = np.ascontiguousarray(X, dtype=np.float64)
            yy = np.ascontiguousarray(y, dtype=np.float64)
            self._keep += [x, yy]
            s.X, s.y, s.n = x.ctypes.data, yy.ctypes.data, x.shape[0]
        self._s = s
        self.theta = float(theta)
        self.params = dict(mean=mean, prec=prec, X=X, y=y, prior_var=prior_var, theta=theta)

    @property
    def ptr(self):
        return C.addressof(self._s)

    def with_theta(self, theta):
        p = dict(self.params)
        p["theta"] = theta
        return Target(self.kind, self.dim, **p)

    def logp(self, x):
        x, px = _d(x)
        return lib().orc_logp(self.ptr, px)

    def grad(self, x):
        x, px = _d(x)
        g = np.empty(self.dim)
        lib().orc_grad(self.ptr, px, _d(g)[1])
        return g

    def hess(self, x):
        x, px = _d(x)
        H = np.empty((self.dim, self.dim))
        lib().orc_hess(self.ptr, px, H.ctypes.data_as(C.POINTER(C.c_double)))
        return H

    def dgrad_dtheta(self, x):
        x, px = _d(x)
        g = np.empty(self.dim)
        lib().orc_dgrad_dtheta(self.ptr, px, g.ctypes.data_as(C.POINTER(C.c_double)))
        return g

    def dlogp_dtheta(self, x):
        x, px = _d(x)
        return lib().orc_dlogp_dtheta(self.ptr, px)


# ------------------------------------------------------------------ chains

def mala_step(tg, eps, x, xi, u, ula=False, force=-1):
    """One MALA/ULA transition (Sec. 3.2).  Returns (x_next, accepted, gtilde, ell, x_prop)."""
    x, px = _d(x)
    xi, pxi = _d(xi)
    out, po = _d(np.empty(tg.dim))
    prop, pp = _d(np.empty(tg.dim))
    gt, ell = C.c_double(), C.c_double()
    a = lib().orc_mala_step(tg.ptr, eps, int(ula), px, pxi, float(u), int(force), po,
                            C.byref(gt), C.byref(ell), pp)
    return out, int(a), gt.value, ell.value, prop


def mala_chain(tg, eps, x0, xi, u, ula=False, force=None):
    """Sequential MALA/ULA chain (Sec. 2 recursion).  Returns (states[T,D], accept[T], gtilde[T])."""
    xi = np.asarray(xi)
    T = xi.shape[0]
    D = tg.dim
    x0, p0 = _d(x0)
    xi, pxi = _d(xi.reshape(T, D))
    if u is None:
        u = np.full(T, 0.5)
    u, pu = _d(u)
    f, pf = _nullable(force, "b")
    st = np.empty((T, D))
    acc = np.empty(T, dtype=np.int8)
    gt = np.empty(T)
    lib().orc_mala_chain(tg.ptr, eps, int(ula), T, p0, pxi, pu, pf, _d(st)[1],
                         acc.ctypes.data_as(C.POINTER(C.c_int8)), _d(gt)[1])
    return st, acc, gt


def mala_jac(tg, eps, x, xi, u, gate=0, ula=False, force=-1):
    """F = f_t(x) and its Jacobian (frozen gate 0, stop-gradient surrogate gate 1)."""
    x, px = _d(x)
    xi, pxi = _d(xi)
    F = np.empty(tg.dim)
    J = np.empty((tg.dim, tg.dim))
    a = lib().orc_mala_jac(tg.ptr, eps, int(ula), int(gate), px, pxi, float(u), int(force),
                           _d(F)[1], J.ctypes.data_as(C.POINTER(C.c_double)))
    return F, J, int(a)


def mala_smoothed_step(tg, eps, x, xi, u):
    x, px = _d(x)
    xi, pxi = _d(xi)
    out = np.empty(tg.dim)
    lib().orc_mala_smoothed_step(tg.ptr, eps, px, pxi, float(u), _d(out)[1])
    return out


def leapfrog_step(tg, eps, s, with_jac=False):
    s, ps = _d(s)
    out = np.empty(2 * tg.dim)
    J = np.empty((2 * tg.dim, 2 * tg.dim)) if with_jac else None
    lib().orc_leapfrog_step(tg.ptr, eps, ps, _d(out)[1],
                            J.ctypes.data_as(C.POINTER(C.c_double)) if with_jac else None)
    return (out, J) if with_jac else out


def hmc_chain(tg, eps, L, x0, momenta, U, force=None, want_traj=False):
    """Sequential HMC, Appendix A.2 algorithm.  Returns dict(chain, accept, logr, s0, traj)."""
    momenta = np.asarray(momenta)
    P = momenta.shape[0]
    D = tg.dim
    x0, p0 = _d(x0)
    m, pm = _d(momenta.reshape(P, D))
    U, pU = _d(U)
    f, pf = _nullable(force, "b")
    chain = np.empty((P + 1, D))
    acc = np.empty(P, dtype=np.int8)
    logr = np.empty(P)
    s0 = np.empty((P, 2 * D))
    traj = np.empty((P, L, 2 * D)) if want_traj else None
    lib().orc_hmc_chain(tg.ptr, eps, int(L), P, p0, pm, pU, pf, _d(chain)[1],
                        acc.ctypes.data_as(C.POINTER(C.c_int8)), _d(logr)[1], _d(s0)[1],
                        traj.ctypes.data_as(C.POINTER(C.c_double)) if want_traj else None)
    return dict(chain=chain, accept=acc, logr=logr, s0=s0, traj=traj)


# ------------------------------------------ HMC across the sequence (Sec. 3.3)

def _mass(inv_mass):
    if inv_mass is None:
        return None, None
    return _d(inv_mass)


def hmc_step(tg, eps, L, x, xi, u, force=-1, inv_mass=None):
    """One whole HMC transition as a chain step f_t (Sec. 3.3, parallel HMC
    across the sequence): momentum xi / sqrt(inv_mass), L leapfrog steps,
    relaxed-gate forward value.  Returns (x_next, accepted, gtilde, H0 - HL, x_L)."""
    x, px = _d(x)
    xi, pxi = _d(xi)
    im, pim = _mass(inv_mass)
    out, po = _d(np.empty(tg.dim))
    prop, pp = _d(np.empty(tg.dim))
    gt, dh = C.c_double(), C.c_double()
    a = lib().orc_hmc_step(tg.ptr, eps, int(L), pim, px, pxi, float(u), int(force), po, C.byref(gt), C.byref(dh), pp)
    return out, int(a), gt.value, dh.value, prop


def hmc_seq_chain(tg, eps, L, x0, xi, u, force=None, inv_mass=None):
    """Sequential chain of HMC transitions.  xi [T, D], u [T].  Returns (states, accept, gtilde)."""
    xi = np.asarray(xi, dtype=np.float64).reshape(-1, tg.dim)
    T = xi.shape[0]
    x0, p0 = _d(x0)
    xi, pxi = _d(xi)
    u, pu = _d(u)
    im, pim = _mass(inv_mass)
    f, pf = _nullable(force, "b")
    st = np.empty((T, tg.dim))
    acc = np.empty(T, dtype=np.int8)
    gt = np.empty(T)
    lib().orc_hmc_seq_chain(tg.ptr, eps, int(L), pim, T, p0, pxi, pu, pf, _d(st)[1],
                            acc.ctypes.data_as(C.POINTER(C.c_int8)), _d(gt)[1])
    return st, acc, gt


def hmc_step_jac(tg, eps, L, x, xi, u, gate=0, force=-1, inv_mass=None):
    """(f_t(x), dense dx_t/dx_{t-1}) of one HMC transition; gate 0 frozen, 1 relaxed."""
    x, px = _d(x)
    xi, pxi = _d(xi)
    im, pim = _mass(inv_mass)
    F, pF = _d(np.empty(tg.dim))
    J, pJ = _d(np.empty((tg.dim, tg.dim)))
    lib().orc_hmc_step_jac(tg.ptr, eps, int(L), pim, int(gate), px, pxi, float(u), int(force), pF, pJ)
    return F, J


def hmc_smoothed_step(tg, eps, L, x, xi, u, inv_mass=None):
    x, px = _d(x)
    xi, pxi = _d(xi)
    im, pim = _mass(inv_mass)
    out, po = _d(np.empty(tg.dim))
    lib().orc_hmc_smoothed_step(tg.ptr, eps, int(L), pim, px, pxi, float(u), po)
    return out


# ------------------------------------------------------- linear recursions

def linrec_diag(a, b):
    """delta_t = a_t delta_{t-1} + b_t (elementwise), delta_0 = 0.  a, b: [T, D]."""
    a, pa = _d(a)
    b, pb = _d(b)
    T, D = b.shape
    out = np.empty((T, D))
    lib().orc_linrec_diag(T, D, pa, pb, _d(out)[1])
    return out


def linrec_dense(A, b):
    """delta_t = A_t delta_{t-1} + b_t, delta_0 = 0.  A: [T, D, D], b: [T, D]."""
    A, pA = _d(A)
    b, pb = _d(b)
    T, D = b.shape
    out = np.empty((T, D))
    lib().orc_linrec_dense(T, D, pA, pb, _d(out)[1])
    return out


def linrec_block2(a, b, c, d, e, f):
    """[p;q]_t = [[a,b],[c,d]]_t [p;q]_{t-1} + [e;f]_t per lane.  All [T, D]."""
    arrs = [_d(v) for v in (a, b, c, d, e, f)]
    T, D = arrs[0][0].shape
    p = np.empty((T, D))
    q = np.empty((T, D))
    lib().orc_linrec_block2(T, D, *[x[1] for x in arrs], _d(p)[1], _d(q)[1])
    return p, q


def bidiagonal_bruteforce(A, b):
    """Solve the same recursion as one (T D) x (T D) block lower-bidiagonal
    system (I - subdiag(A)) delta = b with LAPACK.  For T*D up to ~2000."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    T, D = b.shape
    M = np.eye(T * D)
    for t in range(1, T):
        M[t * D:(t + 1) * D, (t - 1) * D:t * D] = -A[t]
    return np.linalg.solve(M, b.reshape(-1)).reshape(T, D)


# ------------------------------------------------------- derivatives

def mala_tangent(tg, eps, x0, xi, states, accept, dFds, ula=False):
    T, D = states.shape
    out = np.empty(2)
    acc = np.ascontiguousarray(accept, dtype=np.int8)
    lib().orc_mala_tangent(tg.ptr, eps, int(ula), T, _d(x0)[1], _d(np.asarray(xi).reshape(T, D))[1],
                           _d(states)[1], acc.ctypes.data_as(C.POINTER(C.c_int8)), _d(dFds)[1],
                           _d(out)[1])
    return out


def mala_adjoint(tg, eps, x0, xi, states, accept, dFds, ula=False, want_lambda=False):
    T, D = states.shape
    out = np.empty(2)
    acc = np.ascontiguousarray(accept, dtype=np.int8)
    lam = np.empty((T, D)) if want_lambda else None
    x0a, p0 = _d(x0)
    xia, pxi = _d(np.asarray(xi).reshape(T, D))
    sa, ps = _d(states)
    ga, pg = _d(dFds)
    oa, po = _d(out)
    lib().orc_mala_adjoint(tg.ptr, eps, int(ula), T, p0, pxi, ps,
                           acc.ctypes.data_as(C.POINTER(C.c_int8)), pg, po,
                           lam.ctypes.data_as(C.POINTER(C.c_double)) if want_lambda else None)
    return (oa, lam) if want_lambda else oa


# --------------------------------------------- Newton reference (Alg. 1)

_M64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """SplitMix64 (Steele, Lea & Flood 2014): the output function applied to
    x + 0x9E3779B97F4A7C15, all arithmetic modulo 2^64."""
    z = (x + 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def probe_sign(seed: int, sweep: int, t: int, d: int) -> float:
    """Rademacher sign of coordinate d at global step t in sweep `sweep`
    (0-based): -1 if the top bit of m(m(m(seed) ^ sweep) ^ (1024 t + d)) is
    set, else +1, with m = splitmix64."""
    h = splitmix64(splitmix64(splitmix64(seed & _M64) ^ (sweep & _M64)) ^ ((1024 * t + d) & _M64))
    return -1.0 if h >> 63 else 1.0


def hutchinson_diag(J, z):
    """The one-probe estimate z o (J z) of diag(J) (Sec. 3.4 eq. 10): its mean over
    the Rademacher distribution of z is diag(J)."""
    J = np.asarray(J, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    return z * (J @ z)


def damp_and_clip(J, damping=1.0, clip=0.0, inf_norm=False):
    """The damped and clipped Jacobian that full DEER is run with (the paper
    damps full DEER, Sec. 2 and App. A; the two clip forms are this
    project's reading): kappa J, then either every entry clamped to
    [-clip, clip], or the whole matrix scaled by clip / ||kappa J||_inf when
    that row-sum norm exceeds clip.  clip <= 0 leaves kappa J."""
    J = float(damping) * np.asarray(J, dtype=np.float64)
    if clip <= 0:
        return J
    if inf_norm:
        nrm = np.max(np.sum(np.abs(J), axis=1))
        return J * (clip / nrm) if nrm > clip else J
    return np.clip(J, -clip, clip)


def rotated_provider(step_and_jac, Q):
    """The chain in the coordinates z = Q^T s of an orthogonal Q (Sec. 3.4
    eq. 11): z_t = Q^T f_t(Q z_{t-1}) with Jacobian Q^T J_t Q.  Wraps a
    step_and_jac(t, s_prev) provider of newton_reference; its initial state
    must be given as Q^T s_0."""
    Q = np.asarray(Q, dtype=np.float64)

    def sj(t, z_prev):
        F, J = step_and_jac(t, Q @ np.asarray(z_prev, dtype=np.float64))
        return Q.T @ F, Q.T @ J @ Q
    return sj


def _structure(J, variant, D):
    """Project a dense Jacobian onto the variant's structure."""
    if variant == "dense":
        return J
    if variant == "diag":
        return np.diag(np.diag(J))
    if variant == "picard":
        return np.zeros_like(J)
    if variant == "block2":  # diagonal of each D x D block of a 2D x 2D matrix (App. A.3)
        h = D // 2
        out = np.zeros_like(J)
        for bi in range(2):
            for bj in range(2):
                blk = J[bi * h:(bi + 1) * h, bj * h:(bj + 1) * h]
                out[bi * h:(bi + 1) * h, bj * h:(bj + 1) * h] = np.diag(np.diag(blk))
        return out
    raise ValueError(variant)


def block2_probe_jacobian(J, eps, z):
    """Block quasi-DEER Jacobian of a leapfrog step (App. A.3) with the
    Hessian diagonal estimated from one Hessian-vector product: the step's
    Jacobian is [[I, eps I], [eps H, I + eps^2 H]] (s = [x, v], 2D x 2D), so
    H = J[D:, :D] / eps, and h = z o (H z) replaces diag(H) in
    [[I, eps I], [eps diag(h), I + eps^2 diag(h)]]."""
    J = np.asarray(J, dtype=np.float64)
    D = J.shape[0] // 2
    H = J[D:, :D] / eps
    h = np.asarray(z, dtype=np.float64) * (H @ np.asarray(z, dtype=np.float64))
    out = np.zeros_like(J)
    out[:D, :D] = np.eye(D)
    out[:D, D:] = eps * np.eye(D)
    out[D:, :D] = eps * np.diag(h)
    out[D:, D:] = np.eye(D) + eps * eps * np.diag(h)
    return out


def newton_reference(step_and_jac, s0, T, variant="dense", init=None, max_iter=None, tol=0.0,
                     full_trace=True, probe_seed=0, step0=0, jac_transform=None):
    """Algorithm 1 (Appendix A.1) with the update of Sec. 2 eq. 2, in FP64.

    step_and_jac(t, s_prev) -> (f_t(s_prev), df_t/ds(s_prev)) for t = 0..T-1.
    Each sweep linearises every step at the current guess, then solves
    s_t^{new} = f_t(s_{t-1}) + J_t (s_{t-1}^{new} - s_{t-1}) sequentially.
    variant "hutchinson" takes J_t = diag(z o (J z)) with z the probe signs
    of (probe_seed, sweep, step0 + t): step0 is the chain's first global step
    when the chain is one of a batch laid end to end.  Stops when max_t |s^{new}_t - s_t|_inf <= tol,
    or after max_iter sweeps (default T + 1).  jac_transform(J, t, sweep), when
    given, replaces the variant's structure with its own approximate Jacobian
    (e.g. block2_probe_jacobian).  Returns (final trajectory, list of
    iterates, sweeps).
    """
    s0 = np.asarray(s0, dtype=np.float64)
    D = s0.shape[0]
    S = np.tile(s0, (T, 1)) if init is None else np.array(init, dtype=np.float64)
    trace = [S.copy()] if full_trace else []
    max_iter = T + 1 if max_iter is None else max_iter
    it = 0
    while it < max_iter:
        F = np.empty((T, D))
        Js = np.empty((T, D, D))
        for t in range(T):
            prev = s0 if t == 0 else S[t - 1]
            F[t], J = step_and_jac(t, prev)
            if jac_transform is not None:
                Js[t] = jac_transform(J, t, it)
            elif variant == "hutchinson":
                z = np.array([probe_sign(probe_seed, it, step0 + t, d) for d in range(D)])
                Js[t] = np.diag(hutchinson_diag(J, z))
            else:
                Js[t] = _structure(J, variant, D)
        new = np.empty((T, D))
        for t in range(T):
            if t == 0:
                new[t] = F[t]
            else:
                new[t] = F[t] + Js[t] @ (new[t - 1] - S[t - 1])
        delta = np.max(np.abs(new - S)) if T else 0.0
        S = new
        it += 1
        if full_trace:
            trace.append(S.copy())
        if delta <= tol:
            break
    return S, trace, it
