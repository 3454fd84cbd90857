"""ctypes binding of libdgfs.so (argument marshalling only).

Device memory and streams come from PyTorch (``torch.cuda``); every step of
the collision operator runs in the HIP library.  Importing this module loads
the library and raises ImportError if it has not been built
(``python -m paper_1903_04670_amd.build``).
"""
import ctypes as ct
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdgfs.so")
if not os.path.exists(LIB_PATH):
    raise ImportError("libdgfs.so is not built; run python -m paper_1903_04670_amd.build")
lib = ct.CDLL(LIB_PATH)

OK, EINVAL, EUNSUPPORTED, ENOMEM, EHIP, EWORKSPACE, ENONFINITE = 0, -1, -2, -3, -4, -5, -6
FP64, FP32_MIXED = 0, 1
OP_COLLIDE, OP_VJP, OP_RHS, OP_STEP = 0, 1, 2, 3
ACCUMULATE, PROJECT, CHECK, EULER = 0x1, 0x2, 0x4, 0x8
SPHERE_KIND = {"octahedron": 0, "icosahedron": 1, "fibonacci": 2}
MAX_SPECIES = 4

_dp = ct.POINTER(ct.c_double)


class Params(ct.Structure):
    _fields_ = [("n_species", ct.c_int32), ("mass", _dp), ("omega", _dp), ("alpha", _dp),
                ("beta", _dp), ("kn", _dp), ("N", ct.c_int32), ("L", ct.c_double), ("S", ct.c_double),
                ("R", _dp), ("M", ct.c_int32), ("sigma", _dp), ("w_sigma", _dp), ("N_rho", ct.c_int32),
                ("dg_order", ct.c_int32), ("precision", ct.c_int32), ("nyquist_zero", ct.c_int32)]


class Mesh(ct.Structure):
    _fields_ = [("K", ct.c_int32), ("x_left", ct.c_double), ("x_right", ct.c_double),
                ("u_left", ct.c_double * 3), ("T_left", ct.c_double),
                ("u_right", ct.c_double * 3), ("T_right", ct.c_double)]


class Mesh2D(ct.Structure):
    _fields_ = [("Kx", ct.c_int32), ("Ky", ct.c_int32), ("x_left", ct.c_double), ("x_right", ct.c_double),
                ("y_bottom", ct.c_double), ("y_top", ct.c_double), ("periodic_x", ct.c_int32),
                ("periodic_y", ct.c_int32),
                ("u_left", ct.c_double * 3), ("T_left", ct.c_double),
                ("u_right", ct.c_double * 3), ("T_right", ct.c_double),
                ("u_bottom", ct.c_double * 3), ("T_bottom", ct.c_double),
                ("u_top", ct.c_double * 3), ("T_top", ct.c_double)]


class Item(ct.Structure):
    _fields_ = [("plan", ct.c_int32), ("p", ct.c_int32), ("q", ct.c_int32), ("n_nodes", ct.c_int64),
                ("fp", ct.c_void_p), ("fq", ct.c_void_p), ("node_stride", ct.c_int64),
                ("Q", ct.c_void_p), ("out_stride", ct.c_int64)]


_vp, _i32, _i64, _u32, _sz = ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_uint32, ct.c_size_t
lib.dgfs_plan_create.argtypes = [ct.POINTER(Params), ct.POINTER(_vp)]
lib.dgfs_plan_create.restype = ct.c_int
lib.dgfs_plan_destroy.argtypes = [_vp]
lib.dgfs_plan_destroy.restype = None
lib.dgfs_workspace_bytes.argtypes = [_vp, _i64, _i32]
lib.dgfs_workspace_bytes.restype = _sz
lib.dgfs_collide.argtypes = [_vp, _i64, _i32, _i32, _vp, _vp, _i64, _vp, _i64, _u32, _vp, _sz, _vp]
lib.dgfs_collide.restype = ct.c_int
lib.dgfs_collide_noalloc.argtypes = [_vp, _i64, _i32, _i32, _vp, _vp, _i64, _vp, _i64, _u32, _vp]
lib.dgfs_collide_noalloc.restype = ct.c_int
lib.dgfs_collide_vjp.argtypes = [_vp, _i64, _i32, _i32, _vp, _vp, _i64, _vp, _i64, _vp, _vp, _i64, _u32,
                                 _vp, _sz, _vp]
lib.dgfs_collide_vjp.restype = ct.c_int
lib.dgfs_rhs.argtypes = [_vp, ct.POINTER(Mesh), _i64, _vp, _vp, _u32, _vp, _sz, _vp]
lib.dgfs_rhs.restype = ct.c_int
lib.dgfs_step.argtypes = [_vp, ct.POINTER(Mesh), _i64, _vp, ct.c_double, _i32, _u32, _vp, _sz, _vp]
lib.dgfs_step.restype = ct.c_int
lib.dgfs_rhs_2d.argtypes = [_vp, ct.POINTER(Mesh2D), _i64, _vp, _vp, _u32, _vp, _sz, _vp]
lib.dgfs_rhs_2d.restype = ct.c_int
lib.dgfs_step_2d.argtypes = [_vp, ct.POINTER(Mesh2D), _i64, _vp, ct.c_double, _i32, _u32, _vp, _sz, _vp]
lib.dgfs_step_2d.restype = ct.c_int
lib.dgfs_batched_workspace_bytes.argtypes = [ct.POINTER(_vp), _i32, ct.POINTER(Item), _i64]
lib.dgfs_batched_workspace_bytes.restype = _sz
lib.dgfs_collide_batched.argtypes = [ct.POINTER(_vp), _i32, ct.POINTER(Item), _i64, _u32, _vp, _sz, _vp]
lib.dgfs_collide_batched.restype = ct.c_int
lib.dgfs_profile_enable.argtypes = [_i32]
lib.dgfs_profile_enable.restype = ct.c_int
lib.dgfs_profile_read.argtypes = [_i32, ct.c_char_p, ct.POINTER(ct.c_int64), ct.POINTER(ct.c_double)]
lib.dgfs_profile_read.restype = _i32
lib.dgfs_autotune.argtypes = [_vp, _i64, _i32, _i32, _vp, _vp, _i64, _vp, _i64, _vp, _sz, _vp,
                              ct.POINTER(ct.c_int32)]
lib.dgfs_autotune.restype = ct.c_int
lib.dgfs_autotune_rhs.argtypes = [_vp, ct.POINTER(Mesh), _i64, _vp, _vp, _u32, _vp, _sz, _vp, ct.POINTER(ct.c_int32)]
lib.dgfs_autotune_rhs.restype = ct.c_int
lib.dgfs_last_error.argtypes = []
lib.dgfs_last_error.restype = ct.c_char_p
lib.dgfs_sphere_set.argtypes = [_i32, _i32, _dp, _dp]
lib.dgfs_sphere_set.restype = ct.c_int
lib.dgfs_plan_table.argtypes = [_vp, _i32, _i32, _i32, _dp, _i64]
lib.dgfs_plan_table.restype = ct.c_int

EXPORTED = ["dgfs_plan_create", "dgfs_plan_destroy", "dgfs_workspace_bytes", "dgfs_collide",
            "dgfs_collide_vjp", "dgfs_rhs", "dgfs_step", "dgfs_batched_workspace_bytes",
            "dgfs_collide_batched", "dgfs_last_error", "dgfs_sphere_set", "dgfs_plan_table",
            "dgfs_profile_enable", "dgfs_profile_read", "dgfs_autotune", "dgfs_autotune_rhs", "dgfs_rhs_2d",
            "dgfs_step_2d", "dgfs_collide_noalloc"]


def profile_enable(on=True):
    _check(lib.dgfs_profile_enable(1 if on else 0), "dgfs_profile_enable")


def profile_read():
    """{kernel family: (launches, total ms)} recorded since profile_enable."""
    n = lib.dgfs_profile_read(0, None, None, None)
    names = ct.create_string_buffer(64 * max(n, 1))
    counts = (ct.c_int64 * max(n, 1))()
    ms = (ct.c_double * max(n, 1))()
    n = lib.dgfs_profile_read(n, names, counts, ms)
    raw = names.raw
    return {raw[64 * i:64 * i + 64].split(b"\0")[0].decode(): (int(counts[i]), float(ms[i])) for i in range(n)}


class DGFSError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = lib.dgfs_last_error().decode(errors="replace")
        super().__init__("%s failed (status %d): %s" % (where, status, msg))


def _check(status, where):
    if status != OK:
        raise DGFSError(status, where)


def _arr(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).ravel())
    if n is not None and a.size != n:
        raise ValueError("expected %d values, got %d" % (n, a.size))
    return a


def sphere_set(kind, M=None):
    """(sigma [M,3], w [M]) from the library's own sphere sets."""
    k = SPHERE_KIND[kind]
    M = {0: 6, 1: 12}.get(k, M)
    s = np.zeros(3 * M)
    w = np.zeros(M)
    _check(lib.dgfs_sphere_set(k, M, s.ctypes.data_as(_dp), w.ctypes.data_as(_dp)), "dgfs_sphere_set")
    return s.reshape(M, 3), w


class Plan:
    """Immutable plan: species, VSS parameters, grid and quadratures.

    Arguments mirror dgfs_params: masses [ns], omega/alpha [ns, ns],
    N, L, S, sphere (name) or sigma/w_sigma, M, Nrho, optional R/beta/kn
    [ns, ns], dg_order, precision 'fp64' | 'fp32', nyquist_zero (drop the
    Nyquist planes from the gain's translates; not in the paper)."""

    def __init__(self, masses, omega, alpha, N, L, Nrho, sphere="icosahedron", M=None, S=0.0,
                 sigma=None, w_sigma=None, R=None, beta=None, kn=None, dg_order=0, precision="fp64",
                 nyquist_zero=False):
        ns = len(masses)
        self.ns, self.N, self.L, self.Nrho = ns, int(N), float(L), int(Nrho)
        self.masses = [float(m) for m in masses]
        if sigma is None:
            sigma, w_sigma = sphere_set(sphere, M)
        self.sigma = _arr(sigma).reshape(-1, 3)
        self.w_sigma = _arr(w_sigma)
        self.M = len(self.w_sigma)
        self.precision = {"fp64": FP64, "fp32": FP32_MIXED}[precision]
        self.dg_order = int(dg_order)
        self.nyquist_zero = bool(nyquist_zero)
        keep = []

        def ptr(a, n):
            if a is None:
                return None
            v = _arr(a, n)
            keep.append(v)
            return v.ctypes.data_as(_dp)

        p = Params()
        p.n_species = ns
        p.mass = ptr(self.masses, ns)
        p.omega = ptr(omega, ns * ns)
        p.alpha = ptr(alpha, ns * ns)
        p.beta = ptr(beta, ns * ns)
        p.kn = ptr(kn, ns * ns)
        p.N = self.N
        p.L = self.L
        p.S = float(S)
        p.R = ptr(R, ns * ns)
        p.M = self.M
        p.sigma = ptr(self.sigma, 3 * self.M)
        p.w_sigma = ptr(self.w_sigma, self.M)
        p.N_rho = self.Nrho
        p.dg_order = self.dg_order
        p.precision = self.precision
        p.nyquist_zero = int(self.nyquist_zero)
        h = _vp()
        _check(lib.dgfs_plan_create(ct.byref(p), ct.byref(h)), "dgfs_plan_create")
        self.handle = h

    @property
    def n3(self):
        return self.N ** 3

    def close(self):
        if getattr(self, "handle", None):
            lib.dgfs_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def table(self, p, q, which):
        n = {0: self.Nrho, 1: self.Nrho, 2: self.n3, 3: self.Nrho * self.M * self.n3,
             4: self.Nrho * self.M * self.n3, 5: 1}[which]
        out = np.zeros(n)
        _check(lib.dgfs_plan_table(self.handle, p, q, which, out.ctypes.data_as(_dp), n), "dgfs_plan_table")
        return out

    def workspace_bytes(self, n_nodes, op=OP_COLLIDE):
        return int(lib.dgfs_workspace_bytes(self.handle, n_nodes, op))


# ---------------------------------------------------------------- torch glue
def _torch():
    import torch
    return torch


class _Launch:
    """Stream handling of one library call.

    Without an explicit stream the call runs on torch's current stream.
    With a stream `s` other than the current one: `s` first waits for the
    work already queued on the current stream (which produced the inputs);
    buffers the binding allocates (outputs, workspace) are allocated while
    `s` is current, so the caching allocator ties them to `s`; and the
    caller's tensors are recorded on `s`, so their memory is not handed out
    again while `s` still uses it.  Use as a context manager around the
    allocations and the call."""

    def __init__(self, stream, *tensors):
        torch = _torch()
        cur = torch.cuda.current_stream()
        self.side = stream is not None and stream != cur
        self.stream = stream if self.side else cur
        if self.side:
            self.stream.wait_stream(cur)
            for t in tensors:
                if t is not None:
                    t.record_stream(self.stream)
        self._ctx = torch.cuda.stream(self.stream) if self.side else None

    @property
    def ptr(self):
        return ct.c_void_p(self.stream.cuda_stream)

    def __enter__(self):
        if self._ctx is not None:
            self._ctx.__enter__()
        return self

    def __exit__(self, *exc):
        if self._ctx is not None:
            return self._ctx.__exit__(*exc)
        return False


def workspace(plan, n_nodes, op=OP_COLLIDE, device="cuda"):
    torch = _torch()
    n = max(plan.workspace_bytes(n_nodes, op), 256)
    return torch.empty(n, dtype=torch.uint8, device=device)


def _node_view(t, N):
    """(pointer, node stride) of a [n_nodes, ..., N, N, N] float64 cuda tensor
    whose last three dims are contiguous."""
    torch = _torch()
    if t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError("expected a float64 CUDA tensor")
    if tuple(t.shape[-3:]) != (N, N, N) or t.stride(-1) != 1 or t.stride(-2) != N or t.stride(-3) != N * N:
        raise ValueError("last three dims must be a contiguous N^3 block")
    return ct.c_void_p(t.data_ptr()), (t.stride(0) if t.dim() == 4 else N ** 3)


def collide(plan, p, q, fp, fq, out=None, accumulate=False, project=False, check=False, ws=None, stream=None):
    """Q^{pq}(f^p, f^q) for every node: fp, fq, out are [n_nodes, N, N, N]
    float64 CUDA tensors (views with a node stride are fine).  project:
    conservation projection of the result (the mass of species p; for the
    self-collision of one array, p == q and fp is fq, also momentum and
    energy)."""
    torch = _torch()
    if fp.dim() == 3:
        fp, fq = fp[None], fq[None]
        if out is not None:
            out = out[None]
    n_nodes = fp.shape[0]
    if fq.shape[0] != n_nodes:
        raise ValueError("fp and fq node counts differ")
    pf, sf = _node_view(fp, plan.N)
    pq_, sq = _node_view(fq, plan.N)
    if sf != sq and n_nodes > 1:
        raise ValueError("fp and fq must share the node stride")
    with _Launch(stream, fp, fq, out, ws) as run:
        if out is None:
            out = torch.zeros((n_nodes, plan.N, plan.N, plan.N), dtype=torch.float64, device=fp.device)
        po, so = _node_view(out, plan.N)
        if ws is None:
            ws = workspace(plan, n_nodes, OP_COLLIDE, fp.device)
        flags = (ACCUMULATE if accumulate else 0) | (PROJECT if project else 0) | (CHECK if check else 0)
        _check(lib.dgfs_collide(plan.handle, n_nodes, p, q, pf, pq_, sf, po, so, flags,
                                ct.c_void_p(ws.data_ptr()), ws.numel(), run.ptr), "dgfs_collide")
    return out


def collide_noalloc(plan, p, q, fp, fq, out, accumulate=False, project=False, stream=None):
    """dgfs_collide_noalloc: Q^{pq} into `out` with the library's own device
    scratch instead of a workspace (nothing is allocated by the library;
    the caller passes the output).  Calls on one GPU must not overlap."""
    if fp.dim() == 3:
        fp, fq, out = fp[None], fq[None], out[None]
    pf, sf = _node_view(fp, plan.N)
    pq_, sq = _node_view(fq, plan.N)
    po, so = _node_view(out, plan.N)
    if sf != sq and fp.shape[0] > 1:
        raise ValueError("fp and fq must share the node stride")
    flags = (ACCUMULATE if accumulate else 0) | (PROJECT if project else 0)
    with _Launch(stream, fp, fq, out) as run:
        _check(lib.dgfs_collide_noalloc(plan.handle, fp.shape[0], p, q, pf, pq_, sf, po, so, flags, run.ptr),
               "dgfs_collide_noalloc")
    return out


def make_mesh(K, x_left=0.0, x_right=1.0, u_left=(0.0, -0.5, 0.0), T_left=1.0,
              u_right=(0.0, 0.5, 0.0), T_right=1.0):
    m = Mesh()
    m.K = int(K)
    m.x_left, m.x_right = float(x_left), float(x_right)
    m.u_left[:] = [float(v) for v in u_left]
    m.u_right[:] = [float(v) for v in u_right]
    m.T_left, m.T_right = float(T_left), float(T_right)
    return m


def make_mesh2d(Kx, Ky, x=(0.0, 1.0), y=(0.0, 1.0), periodic=(False, True), walls=None):
    """2-D mesh: Kx x Ky rectangles on x[0]..x[1] by y[0]..y[1]; periodic
    (periodic_x, periodic_y); walls {"left"|"right"|"bottom"|"top": (u_w,
    T_w)} for the non-periodic sides."""
    m = Mesh2D()
    m.Kx, m.Ky = int(Kx), int(Ky)
    m.x_left, m.x_right = float(x[0]), float(x[1])
    m.y_bottom, m.y_top = float(y[0]), float(y[1])
    m.periodic_x, m.periodic_y = int(bool(periodic[0])), int(bool(periodic[1]))
    walls = walls or {}
    for side in ("left", "right", "bottom", "top"):
        uw, Tw = walls.get(side, ((0.0, 0.0, 0.0), 1.0))
        getattr(m, "u_" + side)[:] = [float(v) for v in uw]
        setattr(m, "T_" + side, float(Tw))
    return m


def rhs_2d(plan, F, mesh, out=None, project=False, check=False, ws=None, stream=None):
    """dF/dt on a 2-D mesh (transport in x and y + sum_q Q^{pq});
    F [Kx Ky (P+1)^2, ns, N, N, N]."""
    torch = _torch()
    n = _state(plan, F)
    with _Launch(stream, F, out, ws) as run:
        if out is None:
            out = torch.empty_like(F)
        if ws is None:
            ws = workspace(plan, n, OP_RHS, F.device)
        flags = (PROJECT if project else 0) | (CHECK if check else 0)
        _check(lib.dgfs_rhs_2d(plan.handle, ct.byref(mesh), n, ct.c_void_p(F.data_ptr()),
                               ct.c_void_p(out.data_ptr()), flags, ct.c_void_p(ws.data_ptr()), ws.numel(),
                               run.ptr), "dgfs_rhs_2d")
    return out


def step_2d(plan, F, dt, mesh, n_steps=1, project=False, euler=False, check=False, ws=None, stream=None):
    """n_steps SSP-RK3 (or Euler) steps on F in place on a 2-D mesh."""
    n = _state(plan, F)
    with _Launch(stream, F, ws) as run:
        if ws is None:
            ws = workspace(plan, n, OP_STEP, F.device)
        flags = (PROJECT if project else 0) | (EULER if euler else 0) | (CHECK if check else 0)
        _check(lib.dgfs_step_2d(plan.handle, ct.byref(mesh), n, ct.c_void_p(F.data_ptr()), float(dt),
                                int(n_steps), flags, ct.c_void_p(ws.data_ptr()), ws.numel(), run.ptr),
               "dgfs_step_2d")
    return F


def _state(plan, F):
    torch = _torch()
    if F.dtype != torch.float64 or not F.is_cuda or not F.is_contiguous():
        raise TypeError("F must be a contiguous float64 CUDA tensor [n_nodes, ns, N, N, N]")
    if tuple(F.shape[1:]) != (plan.ns, plan.N, plan.N, plan.N):
        raise ValueError("F must have shape [n_nodes, ns, N, N, N]")
    return F.shape[0]


def rhs(plan, F, mesh=None, out=None, project=False, check=False, ws=None, stream=None):
    """dF/dt = DG transport (if mesh) + sum_q Q^{pq}; F [n_nodes, ns, N, N, N]."""
    torch = _torch()
    n = _state(plan, F)
    with _Launch(stream, F, out, ws) as run:
        if out is None:
            out = torch.empty_like(F)
        if ws is None:
            ws = workspace(plan, n, OP_RHS, F.device)
        flags = (PROJECT if project else 0) | (CHECK if check else 0)
        _check(lib.dgfs_rhs(plan.handle, ct.byref(mesh) if mesh is not None else None, n,
                            ct.c_void_p(F.data_ptr()), ct.c_void_p(out.data_ptr()), flags,
                            ct.c_void_p(ws.data_ptr()), ws.numel(), run.ptr), "dgfs_rhs")
    return out


def step(plan, F, dt, n_steps=1, mesh=None, project=False, euler=False, check=False, ws=None, stream=None):
    """n_steps SSP-RK3 (or Euler) steps on F in place."""
    n = _state(plan, F)
    with _Launch(stream, F, ws) as run:
        if ws is None:
            ws = workspace(plan, n, OP_STEP, F.device)
        flags = (PROJECT if project else 0) | (EULER if euler else 0) | (CHECK if check else 0)
        _check(lib.dgfs_step(plan.handle, ct.byref(mesh) if mesh is not None else None, n,
                             ct.c_void_p(F.data_ptr()), float(dt), int(n_steps), flags,
                             ct.c_void_p(ws.data_ptr()), ws.numel(), run.ptr), "dgfs_step")
    return F


def collide_vjp(plan, p, q, fp, fq, wbar, grad_fp=None, grad_fq=None, accumulate=False, ws=None, stream=None):
    """(grad_fp, grad_fq) = ((dQ/df^p)^T wbar, (dQ/df^q)^T wbar) per node;
    all arrays [n_nodes, N, N, N] float64 CUDA tensors (node-strided views ok)."""
    torch = _torch()
    if fp.dim() == 3:
        fp, fq, wbar = fp[None], fq[None], wbar[None]
    n = fp.shape[0]
    pf, sf = _node_view(fp, plan.N)
    pq_, sq = _node_view(fq, plan.N)
    pw, sw = _node_view(wbar, plan.N)
    if n > 1 and sf != sq:
        raise ValueError("fp and fq must share the node stride")
    shape = (n, plan.N, plan.N, plan.N)
    with _Launch(stream, fp, fq, wbar, grad_fp, grad_fq, ws) as run:
        if grad_fp is None:
            grad_fp = torch.zeros(shape, dtype=torch.float64, device=fp.device)
        if grad_fq is None:
            grad_fq = torch.zeros(shape, dtype=torch.float64, device=fp.device)
        pgf, sgf = _node_view(grad_fp, plan.N)
        pgq, sgq = _node_view(grad_fq, plan.N)
        if n > 1 and sgf != sgq:
            raise ValueError("gradients must share the node stride")
        if ws is None:
            ws = workspace(plan, n, OP_VJP, fp.device)
        _check(lib.dgfs_collide_vjp(plan.handle, n, p, q, pf, pq_, sf, pw, sw, pgf, pgq, sgf,
                                    ACCUMULATE if accumulate else 0, ct.c_void_p(ws.data_ptr()), ws.numel(),
                                    run.ptr), "dgfs_collide_vjp")
    return grad_fp, grad_fq


class _CollideFn:
    """torch.autograd.Function wrapper: forward = dgfs_collide, backward =
    dgfs_collide_vjp.  Only (f^p, f^q) are saved; the (r, m) intermediates
    are recomputed in backward."""
    _cls = None

    @classmethod
    def get(cls):
        if cls._cls is None:
            torch = _torch()

            class CollideFunction(torch.autograd.Function):
                @staticmethod
                def forward(ctx, fp, fq, plan, p, q):
                    ctx.plan, ctx.p, ctx.q = plan, p, q
                    ctx.save_for_backward(fp, fq)
                    return collide(plan, p, q, fp.contiguous(), fq.contiguous())

                @staticmethod
                def backward(ctx, g):
                    fp, fq = ctx.saved_tensors
                    gf, gq = collide_vjp(ctx.plan, ctx.p, ctx.q, fp.contiguous(), fq.contiguous(), g.contiguous())
                    return gf, gq, None, None, None
            cls._cls = CollideFunction
        return cls._cls


def collide_autograd(plan, p, q, fp, fq):
    """Differentiable Q^{pq}(fp, fq) for [n_nodes, N, N, N] float64 tensors."""
    return _CollideFn.get().apply(fp, fq, plan, p, q)


class Batch:
    """A heterogeneous batch whose descriptor array is built once.

    plans: list of Plan (same precision); items: list of
    (plan_index, p, q, fp, fq, out) with [n_nodes, N, N, N] float64 CUDA
    tensors (node-strided views allowed).  The batch keeps references to the
    plans and tensors; run() launches dgfs_collide_batched on the arrays as
    they are at that time (one launch per pipeline stage per workspace
    chunk)."""

    def __init__(self, plans, items):
        self.plans = list(plans)
        self.items = list(items)
        self.handles = (ct.c_void_p * len(self.plans))(*[pl.handle for pl in self.plans])
        self.arr = (Item * max(len(self.items), 1))()
        for i, (k, p, q, fp, fq, out) in enumerate(self.items):
            N = self.plans[k].N
            if fp.dim() == 3:
                fp, fq, out = fp[None], fq[None], out[None]
            pf, sf = _node_view(fp, N)
            pq_, sq = _node_view(fq, N)
            po, so = _node_view(out, N)
            if fp.shape[0] > 1 and sf != sq:
                raise ValueError("item %d: fp and fq must share the node stride" % i)
            self.arr[i] = Item(k, p, q, fp.shape[0], pf, pq_, sf, po, so)
        self.tensors = [t for it in self.items for t in it[3:6]]

    def workspace_bytes(self):
        nb = lib.dgfs_batched_workspace_bytes(self.handles, len(self.plans), self.arr, len(self.items))
        if nb == 0 and self.items:
            raise DGFSError(EINVAL, "dgfs_batched_workspace_bytes")
        return max(nb, 256)

    def run(self, accumulate=False, ws=None, stream=None):
        """Launch the batch; returns the workspace used (allocated if None)."""
        torch = _torch()
        with _Launch(stream, ws, *self.tensors) as run:
            if ws is None:
                ws = torch.empty(self.workspace_bytes(), dtype=torch.uint8, device="cuda")
            _check(lib.dgfs_collide_batched(self.handles, len(self.plans), self.arr, len(self.items),
                                            ACCUMULATE if accumulate else 0, ct.c_void_p(ws.data_ptr()),
                                            ws.numel(), run.ptr), "dgfs_collide_batched")
        return ws


def collide_batched(plans, items, accumulate=False, ws=None, stream=None):
    """Heterogeneous batch in one launch per pipeline stage (see Batch);
    returns the workspace used."""
    return Batch(plans, items).run(accumulate=accumulate, ws=ws, stream=stream)


def autotune(plan, p, q, fp, fq, out, ws=None, stream=None):
    """Pick the launch schedule for this plan by timing dgfs_collide on the
    given [n_nodes, N, N, N] inputs; returns (chunk width in evaluations
    per launch or 0 for the default, x-shift split or 0 for the default,
    gain_x fusion 0/1 or -1 for the default).  A dimension leaves its
    default only for a candidate more than 3% faster."""
    torch = _torch()
    n = fp.shape[0]
    pf, sf = _node_view(fp, plan.N)
    pq_, _ = _node_view(fq, plan.N)
    po, so = _node_view(out, plan.N)
    chosen = (ct.c_int32 * 3)()
    with _Launch(stream, fp, fq, out, ws) as run:
        if ws is None:
            # room for the widest candidate
            ws = torch.empty(max(plan.workspace_bytes(n), 256) * 4, dtype=torch.uint8, device=fp.device)
        _check(lib.dgfs_autotune(plan.handle, n, p, q, pf, pq_, sf, po, so, ct.c_void_p(ws.data_ptr()),
                                 ws.numel(), run.ptr, chosen), "dgfs_autotune")
    return tuple(int(v) for v in chosen)


def autotune_rhs(plan, F, mesh=None, project=False, ws=None, stream=None):
    """The same search timing dgfs_rhs on F [n_nodes, ns, N, N, N] (with the
    mesh's transport when given): the schedule for right-hand sides and
    steps of this shape.  Returns (width, split, fusion) as autotune."""
    torch = _torch()
    n = _state(plan, F)
    chosen = (ct.c_int32 * 3)()
    out = torch.empty_like(F)
    with _Launch(stream, F, out, ws) as run:
        if ws is None:
            # room for the widest candidate
            ws = torch.empty(max(plan.workspace_bytes(n, OP_RHS), 256) * 4, dtype=torch.uint8, device=F.device)
        _check(lib.dgfs_autotune_rhs(plan.handle, ct.byref(mesh) if mesh is not None else None, n,
                                     ct.c_void_p(F.data_ptr()), ct.c_void_p(out.data_ptr()),
                                     PROJECT if project else 0, ct.c_void_p(ws.data_ptr()), ws.numel(), run.ptr,
                                     chosen), "dgfs_autotune_rhs")
    return tuple(int(v) for v in chosen)
