"""ctypes binding of libimexdg.so (argument marshalling only).

Every function of include/imexdg.h is exposed under the same name; the Mesh
and Solver classes wrap them with torch tensors supplying device memory and
the current HIP stream. Loading fails loudly when the library is not built:
there is no fallback implementation.
"""
import ctypes
import os

import numpy as np
import torch

from . import workloads as W

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libimexdg.so")

IMX_OK, IMX_EINVAL, IMX_ENOMEM, IMX_EHIP, IMX_ENOCONV, IMX_ENONFINITE, IMX_EREJECT, IMX_ESTATE = range(8)
IMX_R1, IMX_R2 = 1, 2
IMX_FP64, IMX_MIXED = 0, 1

_c_i64p = ctypes.POINTER(ctypes.c_int64)
_c_ip = ctypes.POINTER(ctypes.c_int)
_vp = ctypes.c_void_p


class imx_mesh_desc(ctypes.Structure):
    _fields_ = [("Lx", ctypes.c_double), ("Ly", ctypes.c_double), ("Lz", ctypes.c_double),
                ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int), ("degree", ctypes.c_int),
                ("periodic_x", ctypes.c_int), ("periodic_y", ctypes.c_int), ("terrain", ctypes.c_int),
                ("h0", ctypes.c_double), ("a", ctypes.c_double), ("xc", ctypes.c_double), ("yc", ctypes.c_double),
                ("n_ref", ctypes.c_int), ("ref_boxes", ctypes.POINTER(ctypes.c_double))]


class imx_phys(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("R", ctypes.c_double), ("g", ctypes.c_double), ("f", ctypes.c_double),
                ("sponge_zB", ctypes.c_double), ("sponge_zT", ctypes.c_double), ("sponge_lambda", ctypes.c_double),
                ("sponge_u", ctypes.c_double * 3), ("sponge_xw", ctypes.c_double), ("sponge_yw", ctypes.c_double),
                ("slice", ctypes.c_int)]


class imx_numerics(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("scheme", ctypes.c_int), ("precision", ctypes.c_int),
                ("picard_tol", ctypes.c_double), ("picard_max", ctypes.c_int), ("gmres_tol", ctypes.c_double),
                ("gmres_restart", ctypes.c_int), ("gmres_max", ctypes.c_int), ("fixed_iterations", ctypes.c_int),
                ("inner_tol", ctypes.c_double)]


class imx_solve_stats(ctypes.Structure):
    _fields_ = [("picard_iters", ctypes.c_int), ("gmres_iters", ctypes.c_int),
                ("gmres_relres", ctypes.c_double), ("picard_variation", ctypes.c_double)]


class imx_step_stats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int), ("picard_iters", ctypes.c_int), ("gmres_iters", ctypes.c_int),
                ("mass", ctypes.c_double)]


class imx_member_stats(ctypes.Structure):
    _fields_ = [("steps_done", ctypes.c_int), ("status", ctypes.c_int), ("p50_step_ms", ctypes.c_double),
                ("p99_step_ms", ctypes.c_double), ("mean_step_ms", ctypes.c_double), ("queue_ms", ctypes.c_double),
                ("run_ms", ctypes.c_double), ("gmres_iters", ctypes.c_int64)]


class imx_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("rejected", ctypes.c_int64), ("running", ctypes.c_int64), ("waiting", ctypes.c_int64),
                ("pool_bytes", ctypes.c_size_t), ("pool_bytes_in_use", ctypes.c_size_t),
                ("pool_bytes_peak", ctypes.c_size_t), ("p50_step_ms", ctypes.c_double),
                ("p99_step_ms", ctypes.c_double), ("dof_updates", ctypes.c_double), ("busy_seconds", ctypes.c_double)]


# name -> (restype, argtypes); the exported symbol set of include/imexdg.h
SIGNATURES = {
    "imx_last_error": (ctypes.c_char_p, []),
    "imx_solver_last_error": (ctypes.c_char_p, [_vp]),
    "imx_server_last_error": (ctypes.c_char_p, [_vp]),
    "imx_mesh_create": (ctypes.c_int, [ctypes.POINTER(imx_mesh_desc), ctypes.POINTER(_vp)]),
    "imx_mesh_create_box": (ctypes.c_int, [ctypes.POINTER(imx_mesh_desc), ctypes.POINTER(_vp)]),
    "imx_mesh_info": (ctypes.c_int, [_vp, _c_i64p, _c_ip, _c_i64p, _c_ip]),
    "imx_mesh_node_coords": (ctypes.c_int, [_vp, _vp]),
    "imx_mesh_mass_diag": (ctypes.c_int, [_vp, _vp]),
    "imx_mesh_destroy": (None, [_vp]),
    "imx_solver_create": (ctypes.c_int, [_vp, ctypes.POINTER(imx_phys), ctypes.POINTER(imx_numerics), _vp,
                                         ctypes.POINTER(_vp)]),
    "imx_solver_workspace_bytes": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
    "imx_solver_bind_workspace": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t]),
    "imx_solver_set_numerics": (ctypes.c_int, [_vp, ctypes.POINTER(imx_numerics)]),
    "imx_set_state": (ctypes.c_int, [_vp, _vp]),
    "imx_get_state": (ctypes.c_int, [_vp, _vp]),
    "imx_explicit_residual": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "imx_implicit_setup": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "imx_schur_apply": (ctypes.c_int, [_vp, _vp, _vp]),
    "imx_implicit_solve": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(imx_solve_stats)]),
    "imx_step": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(imx_step_stats)]),
    "imx_total_mass": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double)]),
    "imx_total_mass_noalloc": (ctypes.c_int, [_vp, _vp, _vp]),
    "imx_geo_imbalance": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double)]),
    "imx_solver_set_graphs": (ctypes.c_int, [_vp, ctypes.c_int]),
    "imx_solver_set_sponge_target": (ctypes.c_int, [_vp, _vp]),
    "imx_solver_destroy": (None, [_vp]),
    "imx_solver_timing": (ctypes.c_int, [_vp, ctypes.c_int]),
    "imx_solver_timing_report": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                                ctypes.POINTER(ctypes.c_double), _c_i64p]),
    "imx_server_create": (ctypes.c_int, [_vp, ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(_vp)]),
    "imx_server_submit": (ctypes.c_int, [_vp, ctypes.POINTER(imx_mesh_desc), ctypes.POINTER(imx_phys),
                                         ctypes.POINTER(imx_numerics), _vp, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_uint64)]),
    "imx_server_tick": (ctypes.c_int, [_vp, _c_ip, _c_ip]),
    "imx_server_result": (ctypes.c_int, [_vp, ctypes.c_uint64, _vp, ctypes.POINTER(imx_member_stats)]),
    "imx_server_query": (ctypes.c_int, [_vp, ctypes.POINTER(imx_server_stats)]),
    "imx_server_destroy": (None, [_vp]),
    "imx_server_set_graphs": (ctypes.c_int, [_vp, ctypes.c_int]),
    "imx_transfer_workspace_bytes": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(ctypes.c_size_t)]),
    "imx_transfer_state": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_size_t, _vp, _vp, ctypes.c_int, _vp]),
}

KERNEL_KINDS = ["explicit", "pass1", "pass2", "lambda", "dots", "ortho", "lincomb", "stage", "reduce"]

_lib = None


def lib():
    """Loads the in-tree library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libimexdg.so is not built (run __graft_entry__.build()); "
                               "there is no CPU fallback for the HIP path")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class IMXError(RuntimeError):
    def __init__(self, code, where, msg=None):
        if msg is None:
            msg = lib().imx_last_error().decode(errors="replace")
        super().__init__(f"{where}: status {code}: {msg}")
        self.code = code


def check(code, where, solver=None, server=None):
    """Raises IMXError for a failed call; the message is the object's own last
    error when the call acted on a solver or a server."""
    if code != IMX_OK:
        msg = None
        if solver is not None:
            msg = lib().imx_solver_last_error(solver).decode(errors="replace")
        elif server is not None:
            msg = lib().imx_server_last_error(server).decode(errors="replace")
        raise IMXError(code, where, msg)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _desc(ms: W.MeshSpec):
    boxes = np.ascontiguousarray(np.array(ms.ref_boxes, dtype=np.float64).reshape(-1))
    d = imx_mesh_desc(ms.Lx, ms.Ly, ms.Lz, ms.nx, ms.ny, ms.nz, ms.degree, int(ms.periodic_x), int(ms.periodic_y),
                      int(ms.terrain), ms.h0, ms.a, ms.xc, ms.yc, len(ms.ref_boxes),
                      boxes.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if len(ms.ref_boxes) else None)
    return d, boxes


class Mesh:
    def __init__(self, spec: W.MeshSpec):
        self.spec = spec
        d, self._boxes = _desc(spec)
        h = _vp()
        check(lib().imx_mesh_create(ctypes.byref(d), ctypes.byref(h)), "imx_mesh_create")
        self.h = h
        E, Np, nh, dfm = ctypes.c_int64(), ctypes.c_int(), ctypes.c_int64(), ctypes.c_int()
        check(lib().imx_mesh_info(h, ctypes.byref(E), ctypes.byref(Np), ctypes.byref(nh), ctypes.byref(dfm)),
              "imx_mesh_info")
        self.E, self.Np, self.n_hanging, self.deformed = E.value, Np.value, nh.value, bool(dfm.value)

    def node_coords(self):
        out = np.empty((3, self.E, self.Np))
        check(lib().imx_mesh_node_coords(self.h, out.ctypes.data_as(_vp)), "imx_mesh_node_coords")
        return out

    def mass_diag(self):
        out = np.empty((self.E, self.Np))
        check(lib().imx_mesh_mass_diag(self.h, out.ctypes.data_as(_vp)), "imx_mesh_mass_diag")
        return out

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.imx_mesh_destroy(self.h)
            self.h = None


def phys_struct(p: W.PhysSpec):
    return imx_phys(p.gamma, p.R, p.g, p.f, p.sponge_zB, p.sponge_zT, p.sponge_lam, (ctypes.c_double * 3)(*p.sponge_u),
                    p.sponge_xw, p.sponge_yw, int(p.slice))


def num_struct(n: W.NumSpec, precision=IMX_FP64, inner_tol=1e-3):
    return imx_numerics(n.dt, n.scheme, precision, n.picard_tol, n.picard_max, n.gmres_tol, n.gmres_restart,
                        n.gmres_max, int(n.fixed_iterations), inner_tol)


class Solver:
    """A solver bound to a torch-allocated device workspace on `device`."""

    def __init__(self, mesh: Mesh, phys: W.PhysSpec, num: W.NumSpec, device="cuda:0", precision=IMX_FP64,
                 inner_tol=1e-3):
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device available")
        self.mesh = mesh
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        ph, nm = phys_struct(phys), num_struct(num, precision, inner_tol)
        h = _vp()
        with torch.cuda.device(self.device):
            check(lib().imx_solver_create(mesh.h, ctypes.byref(ph), ctypes.byref(nm),
                                          ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
                  "imx_solver_create")
        self.h = h
        nb = ctypes.c_size_t()
        check(lib().imx_solver_workspace_bytes(h, ctypes.byref(nb)), "imx_solver_workspace_bytes")
        self.workspace = torch.empty(nb.value + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        check(lib().imx_solver_bind_workspace(h, ctypes.c_void_p(base + off), nb.value),
              "imx_solver_bind_workspace")
        self.E, self.Np = mesh.E, mesh.Np

    def _t(self, *shape):
        return torch.empty(shape, dtype=torch.float64, device=self.device)

    def set_numerics(self, num: W.NumSpec, precision=IMX_FP64, inner_tol=1e-3):
        nm = num_struct(num, precision, inner_tol)
        check(lib().imx_solver_set_numerics(self.h, ctypes.byref(nm)), "imx_solver_set_numerics", solver=self.h)

    def set_state(self, q):
        q = torch.as_tensor(q, dtype=torch.float64, device=self.device).contiguous()
        check(lib().imx_set_state(self.h, _ptr(q)), "imx_set_state", solver=self.h)
        self._hold = q

    def get_state(self):
        out = self._t(5, self.E, self.Np)
        check(lib().imx_get_state(self.h, _ptr(out)), "imx_get_state", solver=self.h)
        return out

    def explicit_residual(self, q):
        q = torch.as_tensor(q, dtype=torch.float64, device=self.device).contiguous()
        fNS, fS = self._t(5, self.E, self.Np), self._t(4, self.E, self.Np)
        check(lib().imx_explicit_residual(self.h, _ptr(q), _ptr(fNS), _ptr(fS)), "imx_explicit_residual", solver=self.h)
        return fNS, fS

    def implicit_setup(self, rho_l, p_lag, u_lag):
        ts = [torch.as_tensor(a, dtype=torch.float64, device=self.device).contiguous() for a in (rho_l, p_lag, u_lag)]
        check(lib().imx_implicit_setup(self.h, *[_ptr(t) for t in ts]), "imx_implicit_setup", solver=self.h)
        self.stream.synchronize()

    def schur_apply(self, p):
        p = torch.as_tensor(p, dtype=torch.float64, device=self.device).contiguous()
        out = self._t(self.E, self.Np)
        check(lib().imx_schur_apply(self.h, _ptr(p), _ptr(out)), "imx_schur_apply", solver=self.h)
        return out

    def implicit_solve(self, rho_l, F, G0, p0, u0):
        ts = [torch.as_tensor(a, dtype=torch.float64, device=self.device).contiguous() for a in (rho_l, F, G0, p0, u0)]
        p, u = self._t(self.E, self.Np), self._t(3, self.E, self.Np)
        st = imx_solve_stats()
        code = lib().imx_implicit_solve(self.h, *[_ptr(t) for t in ts], _ptr(p), _ptr(u), ctypes.byref(st))
        check(code, "imx_implicit_solve", solver=self.h)
        return p, u, st

    def step(self, nsteps=1):
        st = imx_step_stats()
        check(lib().imx_step(self.h, int(nsteps), ctypes.byref(st)), "imx_step", solver=self.h)
        return st

    def timing(self, enable):
        check(lib().imx_solver_timing(self.h, int(bool(enable))), "imx_solver_timing", solver=self.h)

    def timing_report(self):
        """{kind: (total_ms, algorithmic_bytes, launches)} since timing was enabled."""
        out = {}
        for k, name in enumerate(KERNEL_KINDS):
            ms, by, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
            check(lib().imx_solver_timing_report(self.h, k, ctypes.byref(ms), ctypes.byref(by), ctypes.byref(n)),
                  "imx_solver_timing_report", solver=self.h)
            out[name] = (ms.value, by.value, n.value)
        return out

    def total_mass(self):
        m = ctypes.c_double()
        check(lib().imx_total_mass(self.h, ctypes.byref(m)), "imx_total_mass", solver=self.h)
        return m.value

    def set_graphs(self, enable):
        check(lib().imx_solver_set_graphs(self.h, int(bool(enable))), "imx_solver_set_graphs", solver=self.h)

    def set_sponge_target(self, q):
        """Damping layers relax the whole state towards q (None: momentum only)."""
        if q is None:
            self._starget = None
            check(lib().imx_solver_set_sponge_target(self.h, None), "imx_solver_set_sponge_target", solver=self.h)
            return
        q = torch.as_tensor(q, dtype=torch.float64, device=self.device).contiguous()
        if tuple(q.shape) != (5, self.E, self.Np):
            raise ValueError(f"sponge target must have shape (5, {self.E}, {self.Np}), got {tuple(q.shape)}")
        self._starget = q   # the library retains the pointer: keep the tensor alive
        check(lib().imx_solver_set_sponge_target(self.h, _ptr(q)), "imx_solver_set_sponge_target", solver=self.h)

    def geo_imbalance(self):
        e = ctypes.c_double()
        check(lib().imx_geo_imbalance(self.h, ctypes.byref(e)), "imx_geo_imbalance", solver=self.h)
        return e.value

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            try:
                self.stream.synchronize()
            except Exception:
                pass
            _lib.imx_solver_destroy(self.h)
            self.h = None


def transfer_state(src: "Mesh", dst: "Mesh", q, device="cuda:0"):
    """Nodal fields q [nf][src.E][Np] (array or device tensor) transferred onto
    the refinement `dst` of the same grid (imx_transfer_state); returns a
    device tensor [nf][dst.E][Np]."""
    dev = torch.device(device)
    q = torch.as_tensor(q, dtype=torch.float64, device=dev).contiguous()
    nf = q.shape[0] if q.dim() == 3 else 1
    nb = ctypes.c_size_t()
    check(lib().imx_transfer_workspace_bytes(src.h, dst.h, ctypes.byref(nb)), "imx_transfer_workspace_bytes")
    ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=dev)
    base = ws.data_ptr()
    off = (-base) % 256
    out = torch.empty((nf, dst.E, dst.Np), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    with torch.cuda.device(dev):
        check(lib().imx_transfer_state(src.h, dst.h, ctypes.c_void_p(base + off), nb.value, _ptr(q), _ptr(out),
                                       int(nf), ctypes.c_void_p(stream.cuda_stream)), "imx_transfer_state")
    stream.synchronize()   # the workspace is released when this returns
    return out if q.dim() == 3 else out[0]


def member_pool_bytes(mesh: Mesh, phys: W.PhysSpec, num: W.NumSpec, precision=IMX_FP64, inner_tol=1e-3):
    """Pool bytes a server member of this configuration takes while it runs:
    the solver workspace plus the device copy of its state, each 256-byte
    aligned."""
    ph, nm = phys_struct(phys), num_struct(num, precision, inner_tol)
    h = _vp()
    check(lib().imx_solver_create(mesh.h, ctypes.byref(ph), ctypes.byref(nm), None, ctypes.byref(h)),
          "imx_solver_create")
    nb = ctypes.c_size_t()
    try:
        check(lib().imx_solver_workspace_bytes(h, ctypes.byref(nb)), "imx_solver_workspace_bytes")
    finally:
        lib().imx_solver_destroy(h)
    return nb.value + ((5 * mesh.E * mesh.Np * 8 + 255) // 256) * 256


class Server:
    """Ensemble server over a torch-allocated device pool of `pool_bytes`
    (the HBM budget); members are (mesh, phys, numerics, q0, nsteps)."""

    def __init__(self, pool_bytes, max_running=4, device="cuda:0"):
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device available")
        self.device = torch.device(device)
        self.pool = torch.empty(int(pool_bytes) + 256, dtype=torch.uint8, device=self.device)
        base = self.pool.data_ptr()
        off = (-base) % 256
        torch.cuda.synchronize(self.device)
        h = _vp()
        with torch.cuda.device(self.device):
            check(lib().imx_server_create(ctypes.c_void_p(base + off), int(pool_bytes), int(max_running),
                                          ctypes.byref(h)), "imx_server_create")
        self.h = h
        self.shapes = {}

    def set_graphs(self, enable):
        check(lib().imx_server_set_graphs(self.h, int(bool(enable))), "imx_server_set_graphs", server=self.h)

    def submit(self, spec: W.MeshSpec, phys: W.PhysSpec, num: W.NumSpec, q0, nsteps, precision=IMX_FP64,
               inner_tol=1e-3):
        d, boxes = _desc(spec)
        ph, nm = phys_struct(phys), num_struct(num, precision, inner_tol)
        q = np.ascontiguousarray(np.asarray(q0, dtype=np.float64))
        rid = ctypes.c_uint64()
        with torch.cuda.device(self.device):
            check(lib().imx_server_submit(self.h, ctypes.byref(d), ctypes.byref(ph), ctypes.byref(nm),
                                          q.ctypes.data_as(_vp), int(nsteps), ctypes.byref(rid)),
                  "imx_server_submit", server=self.h)
        self.shapes[rid.value] = q.shape
        return rid.value

    def tick(self):
        r, w = ctypes.c_int(), ctypes.c_int()
        with torch.cuda.device(self.device):
            check(lib().imx_server_tick(self.h, ctypes.byref(r), ctypes.byref(w)), "imx_server_tick", server=self.h)
        return r.value, w.value

    def result(self, rid):
        """(final state, member stats) or None while the member has not finished."""
        out = np.empty(self.shapes[rid], dtype=np.float64)
        st = imx_member_stats()
        code = lib().imx_server_result(self.h, ctypes.c_uint64(rid), out.ctypes.data_as(_vp), ctypes.byref(st))
        if code == IMX_ESTATE:
            return None
        check(code, "imx_server_result", server=self.h)
        return out, st

    def query(self):
        st = imx_server_stats()
        check(lib().imx_server_query(self.h, ctypes.byref(st)), "imx_server_query", server=self.h)
        return st

    def drain(self, poll_s=0.001):
        import time
        while True:
            r, w = self.tick()
            if r == 0 and w == 0:
                return
            time.sleep(poll_s)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.imx_server_destroy(self.h)
            self.h = None
