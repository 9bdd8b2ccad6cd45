"""ctypes binding of ``libdolinc.so`` (argument marshalling only).

Every compute step runs in the library's HIP kernels; PyTorch supplies device
memory and the stream.  There is no CPU fallback: if the library is missing
or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdolinc.so")

OK, EINVAL, EMESH, ENOMEM, EHIP, ESTATE, EUNSUPPORTED = range(7)
PDE = {"advection": 0, "burgers": 1, "euler": 2}
SCHEME = {"FOU": 1, "CD2": 2, "USR3": 3, "CSR4": 4, "USR5": 5, "ENO3": 6, "WENO5": 7, "CSR6": 8}
FLUX = {"upwind": 0, "rusanov": 1, "hllc": 2}
PRECISION = {"fp64": 0, "fp32": 1}
BLEND = {"none": 0, "theta": 1, "classical": 2, "learned": 3}
MLP_PARAMS = 5825
N_FEATURES = 24
FEATURE_STRIDE = 32
MLP_STATIC_MAX_ROWS = 65536  # dolinc_mlp_train_step_static batch limit


class MeshDesc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_nodes", C.c_int64), ("n_cells", C.c_int64), ("n_faces", C.c_int64),
                ("node_xyz", C.c_void_p), ("face_node_ptr", C.c_void_p), ("face_nodes", C.c_void_p),
                ("owner", C.c_void_p), ("neighbour", C.c_void_p), ("neigh_shift", C.c_void_p),
                ("renumber", C.c_int32), ("part_cells", C.c_int32), ("face_patch", C.c_void_p),
                ("n_patches", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("pde", C.c_int32), ("scheme", C.c_int32), ("flux", C.c_int32), ("precision", C.c_int32),
                ("blend", C.c_int32), ("use_u_ref", C.c_int32), ("gamma", C.c_double),
                ("adv_vel", C.c_double * 3), ("burgers_dir", C.c_double * 3), ("u_ref", C.c_double * 5),
                ("positivity", C.c_int32)]


class MeshStats(C.Structure):
    _fields_ = [("n_parts", C.c_int64), ("n_entries", C.c_int64), ("max_entries", C.c_int64),
                ("max_cell_faces", C.c_int64), ("n_slots", C.c_int64), ("n_rows", C.c_int64),
                ("n_boundary_faces", C.c_int64)]


class DolincError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"dolinc status {status}: {msg}")
        self.status = status


_LIB = None

SIGNATURES = {
    "dolinc_create": [C.POINTER(MeshDesc), C.c_void_p, C.POINTER(C.c_void_p)],
    "dolinc_mesh_prepare": [C.POINTER(MeshDesc), C.c_void_p, C.POINTER(MeshStats)],
    "dolinc_permutation": [C.c_void_p, C.c_void_p],
    "dolinc_stats": [C.c_void_p, C.POINTER(MeshStats)],
    "dolinc_set_boundary": [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p],
    "dolinc_precompute": [C.c_void_p, C.POINTER(Params), C.c_void_p],
    "dolinc_residual": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "dolinc_rk_step": [C.c_void_p, C.c_void_p, C.c_double, C.c_void_p],
    "dolinc_advance": [C.c_void_p, C.c_void_p, C.c_double, C.c_int64, C.c_void_p],
    "dolinc_set_theta": [C.c_void_p, C.c_void_p, C.c_void_p],
    "dolinc_classical_theta": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "dolinc_gradients": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "dolinc_face_states": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "dolinc_geometry": [C.c_void_p] + [C.c_void_p] * 6 + [C.c_void_p],
    "dolinc_diagnostics": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "dolinc_timing": [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p],
    "dolinc_features": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "dolinc_mlp_set": [C.c_void_p, C.c_void_p, C.c_void_p],
    "dolinc_mlp_get": [C.c_void_p, C.c_void_p, C.c_void_p],
    "dolinc_mlp_forward": [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p],
    "dolinc_mlp_train_step": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_float, C.c_void_p, C.c_void_p],
    "dolinc_mlp_train_step_static": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_float, C.c_void_p,
                                     C.c_void_p],
    "dolinc_mlp_gradient": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p],
    "dolinc_destroy": [C.c_void_p],
    "dolinc_last_error": [],
    "dolinc_version": [],
}


def load(path=LIB_PATH):
    """Load the HIP library (raises if it has not been built).

    PyTorch is imported first: its HIP runtime then serves the library too
    (the library's dependency on the runtime resolves to the copy already
    loaded).  Loading the library first would bring in a second runtime,
    and the first device call of one of them would find no device."""
    global _LIB
    if _LIB is not None:
        return _LIB
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} not found: build it with paper_2404_08952_amd/build.py")
    lib = C.CDLL(path)
    for name, args in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int32
    lib.dolinc_destroy.restype = None
    lib.dolinc_last_error.restype = C.c_char_p
    _LIB = lib
    return lib


def _check(lib, st):
    if st != OK:
        raise DolincError(st, lib.dolinc_last_error().decode())


def mesh_desc(mesh, renumber=2, part_cells=0):
    """Fill a MeshDesc from a synth.mesh.Mesh; returns (desc, keepalive)."""
    keep = dict(nodes=np.ascontiguousarray(mesh.nodes, dtype=np.float64),
                fptr=np.ascontiguousarray(mesh.face_ptr, dtype=np.int64),
                fn=np.ascontiguousarray(mesh.face_nodes, dtype=np.int32),
                own=np.ascontiguousarray(mesh.owner, dtype=np.int32),
                nei=np.ascontiguousarray(mesh.neighbour, dtype=np.int32),
                sh=np.ascontiguousarray(mesh.shift, dtype=np.float64))
    patch = getattr(mesh, "patch", None)
    n_patches = 0
    if patch is not None:
        keep["patch"] = np.ascontiguousarray(patch, dtype=np.int32)
        n_patches = int(keep["patch"].max()) + 1 if keep["patch"].size else 0
    d = MeshDesc(mesh.dim, mesh.n_nodes, mesh.n_cells, mesh.n_faces,
                 keep["nodes"].ctypes.data, keep["fptr"].ctypes.data, keep["fn"].ctypes.data,
                 keep["own"].ctypes.data, keep["nei"].ctypes.data, keep["sh"].ctypes.data,
                 renumber, part_cells, keep["patch"].ctypes.data if patch is not None else None, n_patches)
    return d, keep


BC = {"zero_gradient": 0, "dirichlet": 1, "neumann": 2, "slip_wall": 3}


def mesh_prepare(mesh, renumber=2, part_cells=0):
    """Host-only preparation (no device): (new_of_old, stats dict)."""
    lib = load()
    d, _keep = mesh_desc(mesh, renumber, part_cells)
    perm = np.empty(mesh.n_cells, dtype=np.int32)
    st = MeshStats()
    _check(lib, lib.dolinc_mesh_prepare(C.byref(d), perm.ctypes.data, C.byref(st)))
    return perm, {k: getattr(st, k) for k, _ in MeshStats._fields_}


def make_params(pde, scheme, flux="upwind", precision="fp64", blend="none", gamma=1.4,
                adv_vel=(1.0, 0.5, 0.0), burgers_dir=(1.0, 1.0, 0.0), u_ref=None, positivity=False):
    p = Params()
    p.pde = PDE[pde]
    p.scheme = SCHEME[scheme]
    p.flux = FLUX[flux]
    p.precision = PRECISION[precision]
    p.blend = BLEND[blend]
    p.positivity = int(bool(positivity))
    p.gamma = gamma
    for k in range(3):
        p.adv_vel[k] = adv_vel[k] if k < len(adv_vel) else 0.0
        p.burgers_dir[k] = burgers_dir[k] if k < len(burgers_dir) else 0.0
    # u_ref: None (full states), a constant reference state (5 values), or
    # "cell" (each face side's own cell as the reference)
    if u_ref is None:
        p.use_u_ref = 0
    elif isinstance(u_ref, str):
        if u_ref != "cell":
            raise ValueError("u_ref must be None, 5 values or 'cell'")
        p.use_u_ref = 2
    else:
        p.use_u_ref = 1
        for k in range(5):
            p.u_ref[k] = u_ref[k]
    return p


class Solver:
    """A mesh uploaded to the GPU plus one set of scheme parameters.

    Device tensors passed in and out are in the library's internal cell order
    (``perm[old] = new``); use ``to_internal`` / ``to_external``.
    """

    def __init__(self, mesh, pde, scheme, flux="upwind", precision="fp64", blend="none", gamma=1.4,
                 adv_vel=(1.0, 0.5, 0.0), burgers_dir=(1.0, 1.0, 0.0), u_ref=None, renumber=2,
                 part_cells=0, device="cuda:0", positivity=False):
        import torch
        self.torch = torch
        self.lib = load()
        self.device = torch.device(device)
        torch.cuda.set_device(self.device)
        d, keep = mesh_desc(mesh, renumber, part_cells)
        h = C.c_void_p()
        _check(self.lib, self.lib.dolinc_create(C.byref(d), self._stream(), C.byref(h)))
        self.h = h
        del keep
        self.dim = mesh.dim
        self.n_cells = mesh.n_cells
        self.n_faces = mesh.n_faces
        self.perm = np.empty(mesh.n_cells, dtype=np.int32)
        _check(self.lib, self.lib.dolinc_permutation(self.h, self.perm.ctypes.data))
        self.inv = np.empty_like(self.perm)
        self.inv[self.perm] = np.arange(mesh.n_cells, dtype=np.int32)
        st = MeshStats()
        _check(self.lib, self.lib.dolinc_stats(self.h, C.byref(st)))
        self.n_rows = int(st.n_rows)          # device rows: cells, then boundary auxiliary cells
        self.configure(pde, scheme, flux, precision, blend, gamma, adv_vel, burgers_dir, u_ref, positivity)

    def configure(self, pde, scheme, flux="upwind", precision="fp64", blend="none", gamma=1.4,
                  adv_vel=(1.0, 0.5, 0.0), burgers_dir=(1.0, 1.0, 0.0), u_ref=None, positivity=False):
        p = make_params(pde, scheme, flux, precision, blend, gamma, adv_vel, burgers_dir, u_ref, positivity)
        self.pde, self.scheme, self.precision = pde, scheme, precision
        self.nv = self.dim + 2 if pde == "euler" else 1
        self.dtype = self.torch.float64 if precision == "fp64" else self.torch.float32
        _check(self.lib, self.lib.dolinc_precompute(self.h, C.byref(p), self._stream()))

    # -- helpers
    def _stream(self):
        return C.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def _ptr(self, t, shape=None, dtype=None):
        if t is None:
            return None
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("expected a contiguous device tensor")
        if dtype is not None and t.dtype != dtype:
            raise TypeError(f"expected {dtype}, got {t.dtype}")
        if shape is not None and tuple(t.shape) != tuple(shape):
            raise ValueError(f"expected shape {shape}, got {tuple(t.shape)}")
        return C.c_void_p(t.data_ptr())

    def set_boundary(self, patch, kind, values=None):
        """Boundary condition of a patch: kind in BC ("zero_gradient",
        "dirichlet", "neumann", "slip_wall"); values per conserved variable:
        the face values (dirichlet) or outward normal gradients (neumann)."""
        v = None
        if values is not None:
            v = np.ascontiguousarray(np.broadcast_to(np.asarray(values, dtype=np.float64), (self.nv,)))
        _check(self.lib, self.lib.dolinc_set_boundary(self.h, int(patch), BC[kind],
                                                      v.ctypes.data if v is not None else None))

    def empty_state(self):
        return self.torch.empty((self.n_rows, self.nv), dtype=self.dtype, device=self.device)

    def to_internal(self, U):
        """Host array in caller order -> device tensor in internal order."""
        U = np.asarray(U).reshape(self.n_cells, -1)
        out = np.zeros((self.n_rows, U.shape[1]), dtype=U.dtype)   # auxiliary rows: set by the library
        out[self.perm] = U
        return self.torch.from_numpy(np.ascontiguousarray(out)).to(self.device, self.dtype)

    def to_external(self, U):
        """Device tensor in internal order -> host float64 array in caller order."""
        a = U.detach().to("cpu", self.torch.float64).numpy()
        return a[self.perm]

    # -- calls
    def residual(self, U, R=None):
        R = self.empty_state() if R is None else R
        _check(self.lib, self.lib.dolinc_residual(self.h, self._ptr(U, (self.n_rows, self.nv), self.dtype),
                                                  self._ptr(R, (self.n_rows, self.nv), self.dtype),
                                                  self._stream()))
        return R

    def rk_step(self, U, dt):
        _check(self.lib, self.lib.dolinc_rk_step(self.h, self._ptr(U, (self.n_rows, self.nv), self.dtype),
                                                 float(dt), self._stream()))
        return U

    def advance(self, U, dt, n):
        _check(self.lib, self.lib.dolinc_advance(self.h, self._ptr(U, (self.n_rows, self.nv), self.dtype),
                                                 float(dt), int(n), self._stream()))
        return U

    def gradients(self, U, second=False):
        t = self.torch
        G1 = t.empty((self.n_rows, self.nv, self.dim), dtype=self.dtype, device=self.device)
        G2 = t.empty((self.n_rows, self.nv, self.dim * (self.dim + 1) // 2), dtype=self.dtype,
                     device=self.device) if second else None
        _check(self.lib, self.lib.dolinc_gradients(self.h, self._ptr(U), self._ptr(G1), self._ptr(G2),
                                                   self._stream()))
        return (G1, G2) if second else G1

    def face_states(self, U):
        t = self.torch
        mk = lambda: t.empty((self.n_faces, self.nv), dtype=self.dtype, device=self.device)  # noqa: E731
        UL, UR, F = mk(), mk(), mk()
        _check(self.lib, self.lib.dolinc_face_states(self.h, self._ptr(U), self._ptr(UL), self._ptr(UR),
                                                     self._ptr(F), self._stream()))
        return UL, UR, F

    def set_theta(self, theta):
        _check(self.lib, self.lib.dolinc_set_theta(self.h, self._ptr(theta, (self.n_rows,),
                                                                     self.torch.float32), self._stream()))

    def classical_theta(self, U):
        th = self.torch.empty(self.n_rows, dtype=self.torch.float32, device=self.device)
        _check(self.lib, self.lib.dolinc_classical_theta(self.h, self._ptr(U), self._ptr(th), self._stream()))
        return th

    def geometry(self):
        t = self.torch
        f64 = dict(dtype=t.float64, device=self.device)
        V = t.empty(self.n_rows, **f64)
        xc = t.empty((self.n_rows, self.dim), **f64)
        S = t.empty((self.n_faces, self.dim), **f64)
        xf = t.empty((self.n_faces, self.dim), **f64)
        om = t.empty(self.n_faces, **f64)
        g = t.empty(self.n_faces, **f64)
        _check(self.lib, self.lib.dolinc_geometry(self.h, *[self._ptr(x) for x in (V, xc, S, xf, om, g)],
                                                  self._stream()))
        return dict(V=V, xc=xc, S=S, xf=xf, omega=om, g=g)

    def diagnostics(self, U, device=False):
        """Conserved totals, min rho (min u), min p (max u), non-finite count;
        a device tensor with ``device=True``, else copied to the host."""
        out = self.torch.empty(self.nv + 3, dtype=self.torch.float64, device=self.device)
        _check(self.lib, self.lib.dolinc_diagnostics(self.h, self._ptr(U), self._ptr(out), self._stream()))
        return out if device else out.cpu().numpy()

    def timing(self, enable):
        """Start (True) / stop (False) per-kernel HIP-event timing; returns the
        accumulated (ms[4], count[4]) for {grad1, grad2, sensor, flux}."""
        ms = np.zeros(4)
        n = np.zeros(4, dtype=np.int64)
        _check(self.lib, self.lib.dolinc_timing(self.h, int(bool(enable)), ms.ctypes.data, n.ctypes.data))
        return ms, n

    # -- learned indicator
    def features(self, U, fp32=True, bf16=True):
        t = self.torch
        X32 = t.empty((self.n_rows, N_FEATURES), dtype=t.float32, device=self.device) if fp32 else None
        Xb = t.empty((self.n_rows, FEATURE_STRIDE), dtype=t.int16, device=self.device) if bf16 else None
        _check(self.lib, self.lib.dolinc_features(self.h, self._ptr(U), self._ptr(X32), self._ptr(Xb),
                                                  self._stream()))
        return X32, Xb

    def mlp_set(self, params):
        """Network parameters from a host array or a device tensor (float32
        [MLP_PARAMS]); copied on the current stream."""
        if isinstance(params, self.torch.Tensor):
            p = params.detach().to(device=self.device, dtype=self.torch.float32).contiguous()
        else:
            h = np.ascontiguousarray(params, dtype=np.float32)
            if not np.all(np.isfinite(h)):
                raise ValueError("non-finite network parameter")
            p = self.torch.from_numpy(h).to(self.device)
        if p.numel() != MLP_PARAMS:
            raise ValueError(f"expected {MLP_PARAMS} parameters")
        _check(self.lib, self.lib.dolinc_mlp_set(self.h, self._ptr(p), self._stream()))
        self._mlp_src = p  # kept until the next set: the copy is stream-ordered

    def mlp_get(self, device=False):
        p = self.torch.empty(MLP_PARAMS, dtype=self.torch.float32, device=self.device)
        _check(self.lib, self.lib.dolinc_mlp_get(self.h, self._ptr(p), self._stream()))
        return p if device else p.cpu().numpy()

    def mlp_forward(self, Xb):
        th = self.torch.empty(Xb.shape[0], dtype=self.torch.float32, device=self.device)
        _check(self.lib, self.lib.dolinc_mlp_forward(self.h, self._ptr(Xb), Xb.shape[0], self._ptr(th),
                                                     self._stream()))
        return th

    def mlp_train_step(self, Xb, y, lr):
        loss = self.torch.empty(1, dtype=self.torch.float32, device=self.device)
        _check(self.lib, self.lib.dolinc_mlp_train_step(self.h, self._ptr(Xb), self._ptr(y), Xb.shape[0],
                                                        float(lr), self._ptr(loss), self._stream()))
        return loss

    def mlp_train_step_static(self, Xb, y, lr, loss=None):
        """The training step without allocation in the library (its partials in
        the library's fixed device array); ``loss``: a caller-owned device
        float tensor of one element, or None."""
        _check(self.lib, self.lib.dolinc_mlp_train_step_static(
            self.h, self._ptr(Xb), self._ptr(y), Xb.shape[0], float(lr),
            None if loss is None else self._ptr(loss), self._stream()))
        return loss

    def mlp_gradient(self, Xb, y):
        t = self.torch
        g = t.empty(MLP_PARAMS, dtype=t.float32, device=self.device)
        loss = t.empty(1, dtype=t.float32, device=self.device)
        _check(self.lib, self.lib.dolinc_mlp_gradient(self.h, self._ptr(Xb), self._ptr(y), Xb.shape[0],
                                                      self._ptr(g), self._ptr(loss), self._stream()))
        return g, loss

    def stats(self):
        st = MeshStats()
        _check(self.lib, self.lib.dolinc_stats(self.h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in MeshStats._fields_}

    def close(self):
        if getattr(self, "h", None):
            self.lib.dolinc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
