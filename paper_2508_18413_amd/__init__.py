"""Parallel-in-sequence MCMC on AMD Instinct MI355X: Python front end of libpmcmc.

The chain s_t = f_t(s_{t-1}) is solved for all t at once by parallel Newton
iterations (DEER / quasi-DEER), each sweep an evaluation kernel and a
single-pass associative scan in HIP.  This module marshals torch tensors
(device memory, current stream) into the C ABI of include/pmcmc.h; nothing is
computed here.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

from . import _binding as B

__all__ = ["Context", "Target", "solve", "solve_noalloc", "sample_sequential", "linrec_diag", "linrec_block2",
           "linrec_dense", "hmc_sample", "adjoint", "autotune", "ParallelMALA", "B"]

VARIANTS = {"dense": B.PMC_DEER_DENSE, "diag": B.PMC_QDEER_DIAG, "block2": B.PMC_QDEER_BLOCK2,
            "picard": B.PMC_PICARD}
PRODUCTS = {"auto": B.PMC_PRODUCTS_AUTO, "f32": B.PMC_PRODUCTS_F32, "split16": B.PMC_PRODUCTS_SPLIT16,
            "refine": B.PMC_PRODUCTS_REFINE}
KINDS = {"gaussian": B.PMC_TARGET_GAUSSIAN, "banana": B.PMC_TARGET_BANANA,
         "logreg": B.PMC_TARGET_LOGREG, "funnel": B.PMC_TARGET_FUNNEL}


def _torch():
    import torch
    return torch


def _dtype_code(t):
    torch = _torch()
    if t == torch.float64:
        return B.PMC_F64
    if t == torch.float32:
        return B.PMC_F32
    raise TypeError(f"unsupported dtype {t}")


def _ptr(x):
    if x is None:
        return None
    if not x.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if not x.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(x.data_ptr())


class Context:
    """pmc_create / pmc_destroy.  Enqueues on torch's current stream of `device`."""

    def __init__(self, device: int = 0, stream=None):
        torch = _torch()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self._stream = stream
        h = C.c_void_p()
        B.check(B.lib().pmc_create(C.byref(h), device, C.c_void_p(stream.cuda_stream)))
        self.h = h

    def set_stream(self, stream):
        self._stream = stream
        B.check(B.lib().pmc_set_stream(self.h, C.c_void_p(stream.cuda_stream)))

    def set_scan_timing(self, on: bool):
        """pmc_set_scan_timing: time the scan kernel of linrec_diag / linrec_block2."""
        B.check(B.lib().pmc_set_scan_timing(self.h, int(bool(on))))

    def last_scan_ms(self) -> float:
        """pmc_last_scan_ms: kernel time of the most recent timed recursion call."""
        ms = C.c_float()
        B.check(B.lib().pmc_last_scan_ms(self.h, C.byref(ms)))
        return ms.value

    def close(self):
        if getattr(self, "h", None):
            B.lib().pmc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Target:
    """pmc_target_create from a workload target dictionary (arrays copied to the GPU).

    A logistic-regression target may name its matrix-product arithmetic with
    spec["products"]: "auto" (default), "f32", "split16" or "refine"
    (split-FP16 sweeps until each chain meets the tolerance, then FP32-product
    sweeps from its first step until it meets it again); see pmc_products in
    include/pmcmc.h."""

    def __init__(self, ctx: Context, spec: dict, dtype=None):
        torch = _torch()
        dtype = dtype or torch.float32
        self.ctx = ctx
        self.kind = spec["kind"]
        self.dim = int(spec["dim"])
        self.dtype = dtype
        d = B.pmc_target_desc()
        d.kind = KINDS[self.kind]
        d.dim = self.dim
        d.dtype = _dtype_code(dtype)
        dev = f"cuda:{ctx.device}"
        keep = []
        if self.kind == "gaussian":
            m = torch.as_tensor(spec["mean"], dtype=dtype, device=dev).contiguous()
            p = torch.as_tensor(spec["prec"], dtype=dtype, device=dev).contiguous()
            keep += [m, p]
            d.mean, d.prec = m.data_ptr(), p.data_ptr()
        elif self.kind == "logreg":
            X = torch.as_tensor(spec["X"], dtype=dtype, device=dev).contiguous()
            y = torch.as_tensor(spec["y"], dtype=dtype, device=dev).contiguous()
            keep += [X, y]
            d.X, d.y, d.n_data = X.data_ptr(), y.data_ptr(), X.shape[0]
            d.prior_var = float(spec.get("prior_var", 1.0))
            d.products = PRODUCTS[spec.get("products", "auto")]
        elif self.kind == "funnel":
            d.theta = float(spec["theta"])
        torch.cuda.synchronize(ctx.device)
        h = C.c_void_p()
        B.check(B.lib().pmc_target_create(ctx.h, C.byref(d), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            B.lib().pmc_target_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Result:
    states: object
    accept: object
    gtilde: object
    status: int
    sweeps: int
    sweeps_per_chain: list
    n_converged: int
    n_accept: int
    resid_inf: float
    resid_l2: float
    max_ratio: float
    nonfinite: int
    elapsed_ms: float
    trace: object = None
    n_floor: int = 0
    eval_ms: float = 0.0
    scan_ms: float = 0.0
    eval_steps: int = 0
    chain_state: list = None  # per chain: 0 converged, 1 at its rounding floor, 2 max_iter


SAMPLERS = {"mala": B.PMC_SAMPLER_MALA, "ula": B.PMC_SAMPLER_ULA, "hmc": B.PMC_SAMPLER_HMC}


def _problem(target, sampler, eps, s0, noise, uniforms, offsets, init_guess, out, acc, gt, n_leapfrog=0,
             inv_mass=None):
    p = B.pmc_problem()
    p.sampler = SAMPLERS[sampler]
    p.n_leapfrog = int(n_leapfrog)
    p.inv_mass = _ptr(inv_mass)
    p.target = target.h
    p.step_size = float(eps)
    n_chains = s0.shape[0] if s0.dim() == 2 else 1
    p.n_chains = n_chains
    p.n_steps = noise.shape[0]
    keep = None
    if offsets is not None:
        keep = (C.c_int64 * len(offsets))(*[int(v) for v in offsets])
        p.offsets = C.cast(keep, C.POINTER(C.c_int64))
    p.s0, p.noise, p.uniforms = _ptr(s0), _ptr(noise), _ptr(uniforms)
    p.init_guess = _ptr(init_guess)
    p.out_states, p.out_accept, p.out_gtilde = _ptr(out), _ptr(acc), _ptr(gt)
    return p, keep


def _options(dtype, variant="diag", jac_prec="f32", gate="frozen", atol=None, rtol=None,
             max_iter=0, damping=1.0, clip=0.0, clip_inf_norm=False, skip_converged_prefix=True,
             graph_sweeps=0, trace=None, floor_stall=None, profile_kernels=False, jac_probes=0,
             probe_seed=0, basis=None, tie_band=None, window_width=0):
    o = B.pmc_options()
    B.check(B.lib().pmc_default_options(C.byref(o), _dtype_code(dtype)))
    o.variant = VARIANTS[variant]
    o.jac_prec = B.PMC_JAC_BF16 if jac_prec == "bf16" else B.PMC_JAC_F32
    o.gate = B.PMC_GATE_SURROGATE if gate == "surrogate" else B.PMC_GATE_FROZEN
    if atol is not None:
        o.atol = atol
    if rtol is not None:
        o.rtol = rtol
    o.max_iter, o.damping, o.clip = int(max_iter), float(damping), float(clip)
    o.clip_inf_norm, o.skip_converged_prefix = int(clip_inf_norm), int(skip_converged_prefix)
    o.graph_sweeps = int(graph_sweeps)
    if floor_stall is not None:
        o.floor_stall = int(floor_stall)
    if tie_band is not None:
        o.tie_band = float(tie_band)
    o.window_width = int(window_width)
    o.profile_kernels = int(bool(profile_kernels))
    o.jac_probes, o.probe_seed = int(jac_probes), int(probe_seed)
    if basis is not None:
        # device tensor [D, D] in the state dtype, kept alive by the caller
        o.basis = basis.data_ptr()
    if trace is not None:
        o.trace_out = trace.data_ptr()
        o.trace_bytes = trace.numel() * trace.element_size()
    return o


def solve_noalloc(ctx: Context, target: Target, eps, s0, noise, uniforms=None, sampler="mala",
                  offsets=None, init_guess=None, want_trace=False, max_iter=0, out=None, **opts) -> Result:
    """pmc_solve_noalloc: pmc_solve with its workspace in the library's static
    per-device scratch array (no device allocation inside the call).  Output
    tensors are allocated here unless passed in `out` = (states, accept, gtilde)."""
    return solve(ctx, target, eps, s0, noise, uniforms, sampler, offsets, init_guess, want_trace, max_iter,
                 _noalloc=True, _out=out, **opts)


def solve(ctx: Context, target: Target, eps, s0, noise, uniforms=None, sampler="mala",
          offsets=None, init_guess=None, want_trace=False, max_iter=0, _noalloc=False, _out=None,
          n_leapfrog=0, inv_mass=None, **opts) -> Result:
    """pmc_solve: parallel Newton solve of one or more chains.  s0: [B, D] (or [D]);
    noise: [n_steps, D]; uniforms: [n_steps]; offsets: host list [B+1] or None.
    sampler "hmc": whole HMC transitions with n_leapfrog leapfrog steps and the
    optional inverse diagonal mass matrix inv_mass [D] (device tensor)."""
    torch = _torch()
    s0 = s0.reshape(-1, target.dim).contiguous()
    n, D = noise.shape
    dev = noise.device
    if _out is not None:
        out, acc, gt = _out
    else:
        out = torch.empty((n, D), dtype=noise.dtype, device=dev)
        acc = torch.empty(n, dtype=torch.uint8, device=dev)
        gt = torch.empty(n, dtype=torch.float32, device=dev)
    p, keep = _problem(target, sampler, eps, s0, noise, uniforms, offsets, init_guess, out, acc, gt,
                       n_leapfrog, inv_mass)
    trace = None
    if want_trace:
        if max_iter <= 0:
            raise ValueError("want_trace needs an explicit max_iter")
        trace = torch.full((max_iter, n, D), float("nan"), dtype=noise.dtype, device=dev)
    o = _options(noise.dtype, trace=trace, max_iter=max_iter, **opts)
    spc = (C.c_int32 * p.n_chains)()
    cst = (C.c_int8 * p.n_chains)()
    r = B.pmc_result()
    r.sweeps_per_chain = C.cast(spc, C.POINTER(C.c_int32))
    r.chain_state = C.cast(cst, C.POINTER(C.c_int8))
    if _noalloc:
        st = B.check(B.lib().pmc_solve_noalloc(ctx.h, C.byref(p), C.byref(o), C.byref(r)),
                     allow=(B.PMC_NOT_CONVERGED,))
    else:
        st = B.check(B.lib().pmc_solve(ctx.h, C.byref(p), C.byref(o), None, 0, C.byref(r)),
                     allow=(B.PMC_NOT_CONVERGED,))
    del keep
    return Result(out, acc, gt, st, r.sweeps_total, list(spc), r.n_converged, r.n_accept,
                  r.resid_inf, r.resid_l2, r.max_ratio, r.nonfinite, r.elapsed_ms, trace,
                  r.n_floor, r.eval_ms, r.scan_ms, r.eval_steps, list(cst))


def sample_sequential(ctx: Context, target: Target, eps, s0, noise, uniforms=None, sampler="mala",
                      offsets=None, n_leapfrog=0, inv_mass=None) -> Result:
    """pmc_sample_sequential: the same chains evaluated step by step on the GPU."""
    torch = _torch()
    s0 = s0.reshape(-1, target.dim).contiguous()
    n, D = noise.shape
    dev = noise.device
    out = torch.empty((n, D), dtype=noise.dtype, device=dev)
    acc = torch.empty(n, dtype=torch.uint8, device=dev)
    gt = torch.empty(n, dtype=torch.float32, device=dev)
    p, keep = _problem(target, sampler, eps, s0, noise, uniforms, offsets, None, out, acc, gt, n_leapfrog,
                       inv_mass)
    r = B.pmc_result()
    B.check(B.lib().pmc_sample_sequential(ctx.h, C.byref(p), C.byref(r)))
    del keep
    return Result(out, acc, gt, B.PMC_OK, 0, [], p.n_chains, 0, 0.0, 0.0, 0.0, 0, r.elapsed_ms)


def linrec_diag(ctx: Context, a, b):
    """pmc_linrec_diag: a, b [n_lanes, T] -> delta [n_lanes, T]."""
    torch = _torch()
    out = torch.empty_like(b)
    B.check(B.lib().pmc_linrec_diag(ctx.h, _dtype_code(b.dtype), b.shape[0], b.shape[1], _ptr(a),
                                    _ptr(b), _ptr(out)))
    return out


def linrec_block2(ctx: Context, coef, rhs):
    """pmc_linrec_block2: coef [4, n_lanes, T], rhs [2, n_lanes, T] -> [2, n_lanes, T]."""
    torch = _torch()
    out = torch.empty_like(rhs)
    B.check(B.lib().pmc_linrec_block2(ctx.h, rhs.shape[1], rhs.shape[2], _ptr(coef), _ptr(rhs),
                                      _ptr(out)))
    return out


def linrec_dense(ctx: Context, A, b, jac_prec="f32"):
    """pmc_linrec_dense: A [T, D, D], b [T, D] -> delta [T, D]."""
    torch = _torch()
    out = torch.empty_like(b)
    jp = B.PMC_JAC_BF16 if jac_prec == "bf16" else B.PMC_JAC_F32
    B.check(B.lib().pmc_linrec_dense(ctx.h, _dtype_code(b.dtype), jp, b.shape[1], b.shape[0],
                                     _ptr(A), _ptr(b), _ptr(out)))
    return out


def hmc_sample(ctx: Context, target: Target, eps, L, x0, momenta, unif, parallel_leapfrog=True,
               **opts):
    """pmc_hmc_sample: sequential HMC proposals, leapfrog solved in parallel or in sequence."""
    torch = _torch()
    n_prop, D = momenta.shape
    dev = momenta.device
    chain = torch.empty((n_prop + 1, D), dtype=torch.float32, device=dev)
    acc = torch.empty(n_prop, dtype=torch.uint8, device=dev)
    logr = torch.empty(n_prop, dtype=torch.float32, device=dev)
    sweeps = (C.c_int32 * max(n_prop, 1))()
    opts.setdefault("variant", "block2")
    o = _options(torch.float32, **opts)
    r = B.pmc_result()
    st = B.check(B.lib().pmc_hmc_sample(ctx.h, target.h, float(eps), int(L), int(n_prop), _ptr(x0),
                                        _ptr(momenta), _ptr(unif), C.byref(o),
                                        int(bool(parallel_leapfrog)), _ptr(chain), _ptr(acc), _ptr(logr),
                                        C.cast(sweeps, C.POINTER(C.c_int32)), C.byref(r)),
                 allow=(B.PMC_NOT_CONVERGED,))
    return dict(chain=chain, accept=acc, logr=logr, sweeps=list(sweeps)[:n_prop], status=st,
                elapsed_ms=r.elapsed_ms, n_accept=r.n_accept)


def adjoint(ctx: Context, target: Target, eps, s0, noise, uniforms, states, accept, dF_ds,
            sampler="mala"):
    """pmc_adjoint: (dF/dtheta, dF/deps) by the reverse scan over J^T."""
    p, keep = _problem(target, sampler, eps, s0.reshape(1, -1).contiguous(), noise, uniforms, None,
                       None, states, None, None)
    th, ep = C.c_double(), C.c_double()
    B.check(B.lib().pmc_adjoint(ctx.h, C.byref(p), _ptr(states), _ptr(accept), _ptr(dF_ds),
                                C.byref(th), C.byref(ep)))
    del keep
    return th.value, ep.value


def autotune(ctx: Context, target: Target, eps, s0, noise, uniforms, cache_path=None, offsets=None,
             **opts):
    """pmc_autotune: pick the scan tile configuration for this shape."""
    p, keep = _problem(target, "mala", eps, s0.reshape(-1, target.dim).contiguous(), noise, uniforms,
                       offsets, None, noise, None, None)
    o = _options(noise.dtype, **opts)
    B.check(B.lib().pmc_autotune(ctx.h, C.byref(p), C.byref(o),
                                 cache_path.encode() if cache_path else None))
    del keep


def _autograd_function():
    torch = _torch()

    class ParallelMALA(torch.autograd.Function):
        """states = ParallelMALA.apply(theta, eps, ctx, spec, s0, noise, uniforms, solve_kw).

        Forward: pmc_solve of the MALA chain on the target `spec` with its
        parameter theta (the funnel's log-scale) and step size eps.  Backward:
        pmc_adjoint, the reverse scan over transposed step Jacobians at the
        converged trajectory (frozen accept gate), returning dL/dtheta and
        dL/deps for the incoming dL/dstates."""

        @staticmethod
        def forward(fctx, theta, eps, ctx, spec, s0, noise, uniforms, solve_kw):
            tg = Target(ctx, dict(spec, theta=float(theta)))
            r = solve(ctx, tg, float(eps), s0, noise, uniforms, **(solve_kw or {}))
            fctx.save_for_backward(r.states, r.accept)
            fctx.keep = (ctx, tg, float(eps), s0, noise, uniforms, theta.dtype, theta.device)
            return r.states

        @staticmethod
        def backward(fctx, g):
            states, accept = fctx.saved_tensors
            ctx, tg, eps, s0, noise, uniforms, dt, dev = fctx.keep
            dth, deps = adjoint(ctx, tg, eps, s0, noise, uniforms, states, accept, g.contiguous())
            return (torch.tensor(dth, dtype=dt, device=dev), torch.tensor(deps, dtype=dt, device=dev),
                    None, None, None, None, None, None)

    return ParallelMALA


def __getattr__(name):
    if name == "ParallelMALA":
        return _autograd_function()
    raise AttributeError(name)
