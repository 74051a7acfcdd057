"""MI355X-native Walk-on-Spheres operator toolbox (Python face of libwos).

    tb = Toolbox(domain, sites, bnodes, walks=10_000, eps=1e-4, seed=1)
    tb.build()                      # queued on torch's current stream
    A = tb.export("A")              # device tensors
    u, grad_u = tb.apply(fbar, g)   # u = A fbar + H g, grad u = B fbar + K g

`domain` is a dict {"kind": "ball"|"box"|"polygon"|"box_minus_ball",
"dim", "center", "radius", "lo", "hi", "verts"}.  All arithmetic runs in the
HIP kernels of libwos.so; this module marshals arguments.
"""
import ctypes

import numpy as np
import torch

from ._lib import (ENERGIES, EXPORTS, HISD_INIT, HISD_PRECOND, KINDS, PRECISION, PROBLEMS, SOLVE_PRECISION, SOLVERS,
                   TALLY_ACC, TALLY_MODES, WosAdamInfo, WosAdamOpts, WosBuildPlan, WosHisdInfo, WosHisdOpts,
                   WosBuildOpts, WosCoeffs, WosOperatorInfo, WosOperatorOpts, WosDomain, WosError, WosServerOpts,
                   WosSolveInfo, WosToolboxInfo, check, lib)

__all__ = ["Toolbox", "Server", "build_toolbox", "build_plan", "gemm_bf16_nt", "WosError", "lib"]


def _stream_handle(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _domain_struct(domain):
    d = WosDomain()
    d.kind = KINDS[domain["kind"]]
    d.dim = int(domain["dim"])
    for key in ("center", "lo", "hi"):
        if key in domain:
            v = list(domain[key]) + [0.0] * (3 - len(domain[key]))
            getattr(d, key)[:] = [float(t) for t in v]
    d.radius = float(domain.get("radius", 0.0))
    keep = None
    if "verts" in domain:
        keep = np.ascontiguousarray(np.asarray(domain["verts"], dtype=np.float64))
        d.nvert = keep.shape[0]
        d.verts = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return d, keep


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr())


def build_opts(walks, eps, seed=0, precision="f32", max_steps=0, fixed_M=0, volume_samples=0, walks_per_item=0,
               regen_threshold=0, autotune=True, tally="auto", sampler="median3", walker_block=0, tally_acc="auto",
               window_pages=0, window_bpages=0, test_phi=None, test_psi=None):
    """The wos_build_opts structure of include/wos.h.  `test_phi` / `test_psi`
    are float64 numpy arrays (m and p values) that the caller keeps alive
    until the structure has been used."""
    dp = ctypes.POINTER(ctypes.c_double)
    return WosBuildOpts(test_phi=None if test_phi is None else test_phi.ctypes.data_as(dp),
                        test_psi=None if test_psi is None else test_psi.ctypes.data_as(dp),
                        walks_per_site=int(walks), eps=float(eps), max_steps=int(max_steps),
                        fixed_M=int(fixed_M), seed=int(seed), precision=PRECISION[precision],
                        volume_samples=int(volume_samples), walks_per_item=int(walks_per_item),
                        regen_threshold=int(regen_threshold), autotune=1 if autotune else 0,
                        tally_mode=TALLY_MODES[tally], sampler={"median3": 0, "lambert": 1}[sampler],
                        walker_block=int(walker_block), tally_acc=TALLY_ACC[tally_acc],
                        window_pages=int(window_pages), window_bpages=int(window_bpages))


def build_plan(domain, sites, bnodes, walks, eps, vcentres=None, **kw):
    """The host decisions of a build (include/wos.h, wos_toolbox_plan), without
    touching the GPU: tally mode, accumulators, work split, window, LDS bytes
    and the fixed-point bound."""
    sites = np.ascontiguousarray(np.asarray(sites, dtype=np.float64))
    bnodes = np.ascontiguousarray(np.asarray(bnodes, dtype=np.float64))
    vc = None if vcentres is None else np.ascontiguousarray(np.asarray(vcentres, dtype=np.float64))
    dom, keep = _domain_struct(domain)
    opts = build_opts(walks, eps, **kw)
    plan = WosBuildPlan()
    dp = ctypes.POINTER(ctypes.c_double)
    check(lib().wos_toolbox_plan(ctypes.byref(dom), sites.ctypes.data_as(dp), sites.shape[0],
                                 vc.ctypes.data_as(dp) if vc is not None else None,
                                 0 if vc is None else vc.shape[0], bnodes.ctypes.data_as(dp), bnodes.shape[0],
                                 ctypes.byref(opts), ctypes.byref(plan)))
    del keep
    out = {f: getattr(plan, f) for f, _ in plan._fields_}
    out["tally_mode"] = {v: k for k, v in TALLY_MODES.items()}[out["tally_mode"]]
    out["tally_acc"] = {v: k for k, v in TALLY_ACC.items()}[out["tally_acc"]]
    return out


PROBE_OPS = {"fma_f32": 0, "add_u32": 1, "sin_f32": 2, "mul_u32": 3, "mul_wide_u32": 4}


def probe_valu(op, iters=4096, stream=None):
    """Lane operations per second of one vector ALU instruction kind over the
    whole GPU (include/wos.h, wos_probe_valu)."""
    rate = ctypes.c_double()
    check(lib().wos_probe_valu(PROBE_OPS[op], int(iters), ctypes.byref(rate), _stream_handle(stream)))
    return rate.value


def gemm_bf16_nt(X, Y, C=None, alpha=1.0, beta=0.0, stream=None):
    """C = alpha X Y^T + beta C on the matrix cores (include/wos.h,
    wos_gemm_bf16_nt): X (M, K), Y (N, K) torch.bfloat16 device tensors,
    C (M, N) float32 (a new one when None)."""
    if X.dtype != torch.bfloat16 or Y.dtype != torch.bfloat16:
        raise TypeError("X and Y must be bfloat16")
    if X.dim() != 2 or Y.dim() != 2 or X.shape[1] != Y.shape[1] or X.stride(1) != 1 or Y.stride(1) != 1:
        raise ValueError("X (M, K) and Y (N, K) with K contiguous")
    M, K = X.shape
    N = Y.shape[0]
    if C is None:
        C = torch.zeros((M, N), dtype=torch.float32, device=X.device)
    if C.dtype != torch.float32 or tuple(C.shape) != (M, N) or C.stride(1) != 1:
        raise ValueError("C must be float32 (M, N), rows contiguous")
    check(lib().wos_gemm_bf16_nt(M, N, K, float(alpha), _dptr(X), X.stride(0), _dptr(Y), Y.stride(0), float(beta),
                                 _dptr(C), C.stride(0), _stream_handle(stream)))
    return C


class Toolbox:
    """A resident toolbox {x, z, A, B, H, K, lambda} on the current GPU."""

    def __init__(self, domain, sites, bnodes, walks, eps, seed=0, precision="f32", max_steps=0,
                 fixed_M=0, volume_samples=0, walks_per_item=0, regen_threshold=0, autotune=True,
                 tally="auto", vcentres=None, sampler="median3", walker_block=0, tally_acc="auto",
                 window_pages=0, window_bpages=0, test_phi=None, test_psi=None):
        """`sites` are the W centres (the walks start there, n rows); with
        `vcentres` the tally points are binned to a V partition of its own
        (m columns; include/wos.h, wos_toolbox_create_wv), else V = W.
        `tally` is the walker's tally mode ("auto", "lds_rows", "window",
        "hbm"; include/wos.h, wos_build_opts.tally_mode).  With test
        values `test_phi` (m, one per V cell) and `test_psi` (p, one per
        boundary node) the build also keeps each site's per-walk moments of
        the four functionals (export "moments")."""
        self.domain = domain
        self.sites = np.ascontiguousarray(np.asarray(sites, dtype=np.float64))
        self.vcentres = None if vcentres is None else np.ascontiguousarray(np.asarray(vcentres, dtype=np.float64))
        self.bnodes = np.ascontiguousarray(np.asarray(bnodes, dtype=np.float64))
        self.dim = int(domain["dim"])
        self.n = self.sites.shape[0]
        self.m = self.n if self.vcentres is None else self.vcentres.shape[0]
        self.p = self.bnodes.shape[0]
        self.seed = int(seed)
        self.precision = precision
        self.walks = int(walks)
        dom, keep = _domain_struct(domain)
        if (test_phi is None) != (test_psi is None):
            raise ValueError("test_phi and test_psi go together")
        phi = psi = None
        if test_phi is not None:
            phi = np.ascontiguousarray(np.asarray(test_phi, dtype=np.float64).reshape(-1))
            psi = np.ascontiguousarray(np.asarray(test_psi, dtype=np.float64).reshape(-1))
            if phi.shape[0] != self.m or psi.shape[0] != self.p:
                raise ValueError("test_phi needs m values and test_psi p values")
        self.moments = phi is not None
        opts = build_opts(walks, eps, seed, precision, max_steps, fixed_M, volume_samples, walks_per_item,
                          regen_threshold, autotune, tally, sampler, walker_block, tally_acc, window_pages,
                          window_bpages, phi, psi)
        h = ctypes.c_void_p()
        dp = ctypes.POINTER(ctypes.c_double)
        if self.vcentres is None:
            check(lib().wos_toolbox_create(ctypes.byref(dom), self.sites.ctypes.data_as(dp), self.n,
                                           self.bnodes.ctypes.data_as(dp), self.p, ctypes.byref(opts),
                                           ctypes.byref(h)))
        else:
            if self.vcentres.ndim != 2 or self.vcentres.shape[1] != self.dim:
                raise ValueError("vcentres must have shape (m, d)")
            check(lib().wos_toolbox_create_wv(ctypes.byref(dom), self.sites.ctypes.data_as(dp), self.n,
                                              self.vcentres.ctypes.data_as(dp), self.m,
                                              self.bnodes.ctypes.data_as(dp), self.p, ctypes.byref(opts),
                                              ctypes.byref(h)))
        del keep, phi, psi
        self._h = h
        self.dtype = torch.float64 if precision == "f64" else torch.float32

    # -------------------------------------------------------------- build
    def build(self, seed=None, stream=None):
        """Queue a full build (lambda, walks, normalisation) on the stream."""
        s = self.seed if seed is None else int(seed)
        check(lib().wos_toolbox_build(self._h, s, _stream_handle(stream)))
        return self

    def save(self, path):
        """Write the built toolbox to `path` (include/wos.h, wos_toolbox_save)."""
        check(lib().wos_toolbox_save(self._h, str(path).encode()))

    @classmethod
    def load(cls, path, stream=None):
        """A toolbox read from a file written by save() (include/wos.h,
        wos_toolbox_load): the same inputs, options and arrays."""
        h = ctypes.c_void_p()
        check(lib().wos_toolbox_load(str(path).encode(), _stream_handle(stream), ctypes.byref(h)))
        self = cls.__new__(cls)
        self._h = h
        inf = WosToolboxInfo()
        check(lib().wos_toolbox_get_info(h, ctypes.byref(inf)))
        self.dim, self.n, self.m, self.p = inf.dim, inf.n, inf.m, inf.p
        self.precision = "f64" if inf.precision == 1 else "f32"
        self.dtype = torch.float64 if self.precision == "f64" else torch.float32
        self.walks = inf.walks_per_site
        self.domain = None
        self.sites = self.vcentres = self.bnodes = None
        self.seed = 0
        return self

    def set_timing(self, enable=True):
        check(lib().wos_toolbox_set_timing(self._h, 1 if enable else 0))

    def timings(self):
        """Kernel durations (ms) of the last build, from HIP events on its stream."""
        w, v, f = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        check(lib().wos_toolbox_get_timings(self._h, ctypes.byref(w), ctypes.byref(v), ctypes.byref(f)))
        return {"walker_ms": w.value, "volume_ms": v.value, "finalize_ms": f.value}

    def info(self):
        inf = WosToolboxInfo()
        check(lib().wos_toolbox_get_info(self._h, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in inf._fields_}

    # ------------------------------------------------------------- export
    def _shape(self, what):
        n, m, p, d = self.n, self.m, self.p, self.dim
        return {"A": ((n, m), self.dtype), "B": ((d, n, m), self.dtype), "H": ((n, p), self.dtype),
                "K": ((d, n, p), self.dtype), "Hcount": ((n, p), torch.int32),
                "lambda": ((n,), torch.float64), "vcount": ((n,), torch.int64),
                "lambda_v": ((m,), torch.float64), "site_steps": ((n,), torch.int64),
                "moments": ((n, 4 + 4 * d), torch.float64),
                "shadow_v": ((m, (d + 1) * n), torch.int16), "shadow_g": ((p, (d + 1) * n), torch.int16)}[what]

    def export(self, what, stream=None):
        """A copy of one toolbox array as a device tensor (Hcount as int32
        holding the uint32 counts; the BF16 shadows as int16 holding their
        bits, `.view(torch.bfloat16)` reads them)."""
        shape, dt = self._shape(what)
        out = torch.empty(shape, dtype=dt, device="cuda")
        check(lib().wos_toolbox_export(self._h, EXPORTS[what], _dptr(out),
                                       out.numel() * out.element_size(), 1, _stream_handle(stream)))
        return out

    # -------------------------------------------------------------- apply
    def apply(self, fbar, g, grad=True, stream=None):
        """u = A fbar + H g and grad u = B fbar + K g (device float64)."""
        fbar = torch.as_tensor(fbar, dtype=torch.float64, device="cuda").contiguous()
        g = torch.as_tensor(g, dtype=torch.float64, device="cuda").contiguous()
        if fbar.numel() != self.m or g.numel() != self.p:
            raise ValueError("fbar must have m entries and g p entries")
        u = torch.empty(self.n, dtype=torch.float64, device="cuda")
        gu = torch.empty((self.dim, self.n), dtype=torch.float64, device="cuda") if grad else None
        check(lib().wos_apply(self._h, _dptr(fbar), _dptr(g), _dptr(u),
                              _dptr(gu) if grad else ctypes.c_void_p(0), _stream_handle(stream)))
        return u, gu

    # -------------------------------------------------------------- solve
    def solve(self, f, g, kind="linear", A=None, b=None, c=None, kappa=1.0, rcond=1e-3, tol=0.0,
              max_iter=0, max_sweeps=0, solver="tsvd", precision="f64", max_refine=0, refine_tol=0.0,
              stream=None):
        """Solve a Dirichlet problem (see include/wos.h, wos_solve).

        f: (n,) right-hand side at the sites in the convention of `kind`;
        g: (p,) boundary data at the nodes; A (n,d,d), b (n,d), c (n,)
        coefficients at the sites for kind="linear".  Returns
        (u, grad_u, q, info) with device float64 tensors."""
        f, g, A, b, c, co = self._coeffs(f, g, kind, A, b, c, kappa, rcond, tol, max_iter, max_sweeps, solver,
                                         precision, max_refine, refine_tol)
        u = torch.empty(self.n, dtype=torch.float64, device="cuda")
        gu = torch.empty((self.dim, self.n), dtype=torch.float64, device="cuda")
        q = torch.empty(self.m, dtype=torch.float64, device="cuda")
        info = WosSolveInfo()
        check(lib().wos_solve(self._h, ctypes.byref(co), _dptr(f), _dptr(g), _dptr(u), _dptr(gu), _dptr(q),
                              ctypes.byref(info), _stream_handle(stream)))
        return u, gu, q, {k: getattr(info, k) for k, _ in info._fields_}

    def solve_noalloc(self, f, g, u, grad_u, q, A=None, b=None, c=None, rcond=1e-3, stream=None):
        """The FP64 Tikhonov solve of a linear problem into caller-provided
        outputs u (n,), grad_u (d, n) or None, q (m,) or None, with the
        library's fixed work array (include/wos.h, wos_solve_noalloc): no
        device allocation by the library.  Returns the info dict."""
        f, g, A, b, c, co = self._coeffs(f, g, "linear", A, b, c, 1.0, rcond, 0.0, 0, 0, "tikhonov", "f64", 0, 0.0)
        info = WosSolveInfo()
        null = ctypes.c_void_p(0)
        check(lib().wos_solve_noalloc(self._h, ctypes.byref(co), _dptr(f), _dptr(g), _dptr(u),
                                      _dptr(grad_u) if grad_u is not None else null,
                                      _dptr(q) if q is not None else null, ctypes.byref(info),
                                      _stream_handle(stream)))
        return {k: getattr(info, k) for k, _ in info._fields_}

    def make_bf16(self, stream=None):
        """Make (or remake) the BF16 shadows of the built toolbox (include/wos.h,
        wos_toolbox_make_bf16)."""
        check(lib().wos_toolbox_make_bf16(self._h, _stream_handle(stream)))
        return self

    def apply_bf16(self, fbar, g, stream=None):
        """wos_apply from the BF16 shadows: (u, grad_u) device float64 tensors."""
        fbar = torch.as_tensor(fbar, dtype=torch.float64, device="cuda").contiguous()
        g = torch.as_tensor(g, dtype=torch.float64, device="cuda").contiguous()
        if fbar.numel() != self.m or g.numel() != self.p:
            raise ValueError("fbar must have m entries and g p entries")
        u = torch.empty(self.n, dtype=torch.float64, device="cuda")
        gu = torch.empty((self.dim, self.n), dtype=torch.float64, device="cuda")
        check(lib().wos_apply_bf16(self._h, _dptr(fbar), _dptr(g), _dptr(u), _dptr(gu), _stream_handle(stream)))
        return u, gu

    def take(self, other, estimators, stream=None):
        """Copy the estimators named in `estimators` (any of "A", "B", "H",
        "K") from `other`, a toolbox built on the same domain, sites and
        nodes with its own walks, fixed_M, eps and seed (include/wos.h,
        wos_toolbox_take): per-estimator (M, N)."""
        bits = {"A": 1, "B": 2, "H": 4, "K": 8}
        mask = 0
        for e in estimators:
            mask |= bits[e]
        check(lib().wos_toolbox_take(self._h, other._h, mask, _stream_handle(stream)))

    def interpolate(self, u, x, grad_u=None, stream=None):
        """u at arbitrary points x (npts, d) of the domain (include/wos.h,
        wos_interpolate): the nearest site's value, plus <grad u_i, x - x_i>
        when grad_u (d, n) is given.  Returns (values, site indices) as
        device tensors."""
        dev = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda").contiguous()
        u, x = dev(u), dev(x)
        if u.numel() != self.n or (x.numel() and x.shape[-1] != self.dim):
            raise ValueError("u must have n entries and x shape (npts, d)")
        gu = None if grad_u is None else dev(grad_u)
        if gu is not None and gu.numel() != self.dim * self.n:
            raise ValueError("grad_u must have d x n entries")
        npts = x.numel() // self.dim
        out = torch.empty(npts, dtype=torch.float64, device="cuda")
        site = torch.empty(npts, dtype=torch.int32, device="cuda")
        check(lib().wos_interpolate(self._h, _dptr(u), _dptr(gu) if gu is not None else ctypes.c_void_p(0),
                                    _dptr(x), npts, _dptr(out), _dptr(site), _stream_handle(stream)))
        return out, site

    def minimize(self, f, g, p_exp, alpha, max_iter, fbar0=1.0, tol=0.0, check_every=0, beta1=-1.0, beta2=-1.0,
                 eps=0.0, energy="plaplace", coef_A=None, coef_c=None, coef_w=None, graph=False, stream=None):
        """Adam on the discrete functional J of the Euler-Lagrange route
        (include/wos.h, wos_minimize), from the source fbar0 (a scalar for a
        constant start, or an (m,) array); energy is "plaplace" (exponent
        p_exp), "minimal_surface", "semilinear" or "elliptic" (with the
        per-site coefficient fields coef_A (n, d, d), coef_c (n,), coef_w
        (n,), each optional; p_exp unused).  graph=True replays the
        iterations between checks as one captured HIP graph.  Returns (u,
        grad_u, fbar, info) with device float64 tensors."""
        dev = lambda x: torch.as_tensor(x, dtype=torch.float64, device="cuda").contiguous()
        f, g = dev(f), dev(g)
        if f.numel() != self.n or g.numel() != self.p:
            raise ValueError("f must have n entries and g p entries")
        if np.ndim(fbar0) == 0:
            fbar = torch.full((self.m,), float(fbar0), dtype=torch.float64, device="cuda")
        else:
            fbar = dev(fbar0).clone()
            if fbar.numel() != self.m:
                raise ValueError("fbar0 must have m entries")
        co = {}
        for key, val, shape in (("coef_A", coef_A, (self.n, self.dim, self.dim)), ("coef_c", coef_c, (self.n,)),
                                ("coef_w", coef_w, (self.n,))):
            if val is not None:
                co[key] = dev(val)
                if tuple(co[key].shape) != shape:
                    raise ValueError("%s must have shape %s" % (key, shape))
        opts = WosAdamOpts(energy=ENERGIES[energy], p_exp=float(p_exp), alpha=float(alpha), beta1=float(beta1),
                           beta2=float(beta2), eps=float(eps), max_iter=int(max_iter), tol=float(tol),
                           check_every=int(check_every), graph=1 if graph else 0,
                           **{k: ctypes.c_void_p(v.data_ptr()) for k, v in co.items()})
        u = torch.empty(self.n, dtype=torch.float64, device="cuda")
        gu = torch.empty((self.dim, self.n), dtype=torch.float64, device="cuda")
        info = WosAdamInfo()
        check(lib().wos_minimize(self._h, ctypes.byref(opts), _dptr(f), _dptr(g), _dptr(fbar), _dptr(u), _dptr(gu),
                                 ctypes.byref(info), _stream_handle(stream)))
        return u, gu, fbar, {k: getattr(info, k) for k, _ in info._fields_}

    def saddle(self, f, g, k, eta, tau, max_iter, fbar0=1.0, V0=None, precond="A", energy="semilinear", p_exp=0.0,
               tol=0.0, check_every=0, graph=False, stream=None):
        """p-HiSD saddle search on J (include/wos.h, wos_saddle) from the
        source fbar0 (scalar or (m,) array) with k directions: V0 (k, m) if
        given, else the eigenvectors of the k smallest eigenvalues of the
        Hessian at fbar0.  precond is "A" (the paper's M = A) or "identity".
        graph=True replays blocks of iterations from one captured HIP graph.
        Returns (u, grad_u, fbar, V, info) with device float64 tensors."""
        dev = lambda x: torch.as_tensor(x, dtype=torch.float64, device="cuda").contiguous()
        f, g = dev(f), dev(g)
        if f.numel() != self.n or g.numel() != self.p:
            raise ValueError("f must have n entries and g p entries")
        if np.ndim(fbar0) == 0:
            fbar = torch.full((self.m,), float(fbar0), dtype=torch.float64, device="cuda")
        else:
            fbar = dev(fbar0).clone()
            if fbar.numel() != self.m:
                raise ValueError("fbar0 must have m entries")
        if not 1 <= int(k) <= 8:
            raise ValueError("k must be in 1..8")
        if V0 is None:
            V = torch.zeros((int(k), self.m), dtype=torch.float64, device="cuda")
        else:
            V = dev(V0).clone()
            if tuple(V.shape) != (int(k), self.m):
                raise ValueError("V0 must have shape (k, m)")
        opts = WosHisdOpts(energy=ENERGIES[energy], p_exp=float(p_exp), k=int(k), eta=float(eta), tau=float(tau),
                           max_iter=int(max_iter), tol=float(tol), check_every=int(check_every),
                           precond=HISD_PRECOND[precond], init=HISD_INIT["given" if V0 is not None else "hessian"],
                           graph=1 if graph else 0)
        u = torch.empty(self.n, dtype=torch.float64, device="cuda")
        gu = torch.empty((self.dim, self.n), dtype=torch.float64, device="cuda")
        info = WosHisdInfo()
        check(lib().wos_saddle(self._h, ctypes.byref(opts), _dptr(f), _dptr(g), _dptr(fbar), _dptr(V), _dptr(u),
                               _dptr(gu), ctypes.byref(info), _stream_handle(stream)))
        return u, gu, fbar, V, {k_: getattr(info, k_) for k_, _ in info._fields_}

    def operator(self, A=None, b=None, c=None, rcond=1e-3, grad=False, storage="f64", stream=None):
        """Prepare the solution operator of the linear problem with these
        coefficients (include/wos.h, wos_operator_create): Tikhonov inverse
        with `rcond`, stored in `storage` ("f64" or "f32")."""
        return Operator(self, A, b, c, rcond, grad, storage, stream)

    def _coeffs(self, f, g, kind="linear", A=None, b=None, c=None, kappa=1.0, rcond=1e-3, tol=0.0, max_iter=0,
                max_sweeps=0, solver="tsvd", precision="f64", max_refine=0, refine_tol=0.0):
        """Device copies of the problem data and the wos_coeffs struct."""
        dev = lambda x: None if x is None else torch.as_tensor(x, dtype=torch.float64, device="cuda").contiguous()
        f, g, A, b, c = dev(f), dev(g), dev(A), dev(b), dev(c)
        if f.numel() != self.n or g.numel() != self.p:
            raise ValueError("f must have n entries and g p entries")
        d = self.dim
        for name, x, size in (("A", A, self.n * d * d), ("b", b, self.n * d), ("c", c, self.n)):
            if x is not None and x.numel() != size:
                raise ValueError("%s must have %d entries (sites x its shape)" % (name, size))
        co = WosCoeffs(kind=PROBLEMS[kind], A=None if A is None else A.data_ptr(),
                       b=None if b is None else b.data_ptr(), c=None if c is None else c.data_ptr(),
                       kappa=float(kappa), rcond=float(rcond), tol=float(tol), max_iter=int(max_iter),
                       max_sweeps=int(max_sweeps), solver=SOLVERS[solver], precision=SOLVE_PRECISION[precision],
                       max_refine=int(max_refine), refine_tol=float(refine_tol))
        return f, g, A, b, c, co

    def free(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().wos_toolbox_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Operator:
    """A prepared solution operator u = U_f f + U_g g (and grad u) of one
    toolbox and one set of linear coefficients."""

    def __init__(self, tb, A, b, c, rcond, grad, storage, stream):
        zf = torch.zeros(tb.n, dtype=torch.float64, device="cuda")
        zg = torch.zeros(tb.p, dtype=torch.float64, device="cuda")
        _, _, A, b, c, co = tb._coeffs(zf, zg, "linear", A, b, c, rcond=rcond, solver="tikhonov")
        opts = WosOperatorOpts(want_grad=1 if grad else 0, storage=PRECISION[storage])
        self._h = ctypes.c_void_p()
        check(lib().wos_operator_create(tb._h, ctypes.byref(co), ctypes.byref(opts), _stream_handle(stream),
                                        ctypes.byref(self._h)))
        self.tb = tb  # the toolbox must outlive the operator
        self.n, self.p, self.dim, self.grad = tb.n, tb.p, tb.dim, bool(grad)

    def info(self):
        inf = WosOperatorInfo()
        check(lib().wos_operator_get_info(self._h, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in inf._fields_}

    def apply(self, f, g, grad=False, stream=None):
        """f (nrhs, n) and g (nrhs, p), or single vectors; returns u (nrhs, n)
        and grad_u (nrhs, d, n) or None, float64 on the device."""
        dev = lambda x: torch.as_tensor(x, dtype=torch.float64, device="cuda").contiguous()
        f, g = dev(f), dev(g)
        single = f.dim() == 1
        f, g = f.reshape(-1, self.n), g.reshape(-1, self.p)
        if f.shape[0] != g.shape[0]:
            raise ValueError("f and g must hold the same number of right-hand sides")
        k = f.shape[0]
        u = torch.empty((k, self.n), dtype=torch.float64, device="cuda")
        gu = torch.empty((k, self.dim, self.n), dtype=torch.float64, device="cuda") if grad else None
        arr = lambda ts: (ctypes.c_void_p * k)(*[t.data_ptr() for t in ts])
        check(lib().wos_operator_apply(self._h, k, arr(f), arr(g), arr(u), arr(gu) if grad else None,
                                       _stream_handle(stream)))
        if single:
            return u[0], (gu[0] if grad else None)
        return u, gu

    def free(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().wos_operator_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Server:
    """Request server over resident toolboxes (include/wos.h, wos_server_*):
    up to `slots` solves run concurrently, each on its own stream."""

    def __init__(self, slots=4, mem_budget=0, max_batch=0):
        self._h = ctypes.c_void_p()
        opts = WosServerOpts(slots=int(slots), mem_budget=int(mem_budget), max_batch=int(max_batch))
        check(lib().wos_server_create(ctypes.byref(opts), ctypes.byref(self._h)))
        self._live = {}  # ticket -> tensors that must outlive the request

    def submit(self, tb, f, g, u=None, grad=False, **problem):
        """Queue a solve on toolbox `tb` (keyword arguments as Toolbox.solve);
        returns (ticket, u, grad_u) with the output tensors it will fill."""
        f, g, A, b, c, co = tb._coeffs(f, g, **problem)
        if u is None:
            u = torch.empty(tb.n, dtype=torch.float64, device="cuda")
        gu = torch.empty((tb.dim, tb.n), dtype=torch.float64, device="cuda") if grad else None
        t = ctypes.c_uint64()
        check(lib().wos_server_submit(self._h, tb._h, ctypes.byref(co), _dptr(f), _dptr(g), _dptr(u),
                                      _dptr(gu) if grad else ctypes.c_void_p(0), ctypes.byref(t)))
        self._live[t.value] = (f, g, A, b, c, u, gu)
        return t.value, u, gu

    def submit_op(self, op, f, g, u=None, grad=False):
        """Queue a solve with a prepared operator; returns (ticket, u, grad_u)."""
        dev = lambda x: torch.as_tensor(x, dtype=torch.float64, device="cuda").contiguous()
        f, g = dev(f), dev(g)
        if f.numel() != op.n or g.numel() != op.p:
            raise ValueError("f must have n entries and g p entries")
        if u is None:
            u = torch.empty(op.n, dtype=torch.float64, device="cuda")
        gu = torch.empty((op.dim, op.n), dtype=torch.float64, device="cuda") if grad else None
        t = ctypes.c_uint64()
        check(lib().wos_server_submit_op(self._h, op._h, _dptr(f), _dptr(g), _dptr(u),
                                         _dptr(gu) if grad else ctypes.c_void_p(0), ctypes.byref(t)))
        self._live[t.value] = (op, f, g, u, gu)
        return t.value, u, gu

    def poll(self, ticket, block=True):
        """None while running (block=False); else (info, (t_submit, t_start, t_end))."""
        info = WosSolveInfo()
        times = (ctypes.c_double * 3)()
        st = lib().wos_server_poll(self._h, ctypes.c_uint64(ticket), 1 if block else 0, ctypes.byref(info), times)
        if st == -6 and not block:
            return None
        self._live.pop(ticket, None)
        check(st)
        return {k: getattr(info, k) for k, _ in info._fields_}, tuple(times)

    def pending(self):
        q, u = ctypes.c_int64(), ctypes.c_int64()
        check(lib().wos_server_pending(self._h, ctypes.byref(q), ctypes.byref(u)))
        return q.value, u.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().wos_server_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_toolbox(domain, sites, bnodes, walks, eps, seed, **kw):
    """build_toolbox(domain, sites, bnodes, walks, eps, seed): create, build
    and wait."""
    tb = Toolbox(domain, sites, bnodes, walks, eps, seed=seed, **kw)
    tb.build()
    torch.cuda.current_stream().synchronize()
    return tb
