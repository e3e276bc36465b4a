"""ctypes binding of the amrto C ABI (``include/amrto.h``).

Argument marshalling only: device buffers are torch tensors on the HIP device
(their ``data_ptr()`` is passed through), host arrays are numpy arrays.  Every
computation happens inside ``libamrto.so``; if the library has not been built
the loader raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libamrto.so")

FP64, FP32, BF16 = 0, 1, 2
JACOBI, BLOCK3 = 0, 1  # preconditioners of Context.pcg
FILTER_SENSITIVITY, FILTER_DENSITY = 0, 1
STATUS = {0: "OK", 1: "NOT_CONVERGED", -1: "EINVAL", -2: "EHIP", -3: "ENOMEM", -4: "EBREAKDOWN", -5: "ESTATE"}

_p = C.c_void_p
_i32p = C.POINTER(C.c_int32)


class AmrtoError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class MeshStruct(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_elems", C.c_int32), ("dims", C.c_int32 * 3),
                ("max_level", C.c_int32), ("node_xyz", _p), ("elem_nodes", _p), ("elem_level", _p),
                ("n_hang", C.c_int32), ("hang_node", _p), ("hang_ptr", _p), ("hang_master", _p),
                ("hang_w", _p), ("dof_fixed", _p)]


class Mesh2DStruct(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_elems", C.c_int32), ("dims", C.c_int32 * 2),
                ("max_level", C.c_int32), ("node_xy", _p), ("elem_nodes", _p), ("elem_level", _p),
                ("n_hang", C.c_int32), ("hang_node", _p), ("hang_ptr", _p), ("hang_master", _p),
                ("hang_w", _p), ("dof_fixed", _p)]


class Region(C.Structure):
    _fields_ = [("has", C.c_int32 * 3), ("at", C.c_int32 * 3)]


class SolveOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("max_it", C.c_int32), ("precond", C.c_int32),
                ("inner_prec", C.c_int32), ("inner_rtol", C.c_double), ("check_every", C.c_int32),
                ("use_coarse", C.c_int32), ("fallback_fp64", C.c_int32), ("single_reduction", C.c_int32),
                ("record", C.c_int32)]


class MgOpts(C.Structure):
    _fields_ = [("degree", C.c_int32), ("ratio", C.c_double), ("power_its", C.c_int32), ("hi_factor", C.c_double),
                ("coarse_dofs", C.c_int32), ("first", C.c_int32), ("coarse_degree", C.c_int32),
                ("blocks0", C.c_int32)]


class SolveStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("outer", C.c_int32), ("rel_res", C.c_double), ("ms", C.c_double),
                ("fell_back", C.c_int32)]


_SIGS = {
    "amrto_create": (C.c_int, [C.POINTER(_p), C.c_int, _p]),
    "amrto_destroy": (C.c_int, [_p]),
    "amrto_last_error": (C.c_char_p, [_p]),
    "amrto_set_stream": (C.c_int, [_p, _p]),
    "amrto_set_deterministic": (C.c_int, [_p, C.c_int32]),
    "amrto_set_material": (C.c_int, [_p, C.c_double, C.c_double, C.c_double, C.c_double]),
    "amrto_upload_mesh": (C.c_int, [_p, C.POINTER(MeshStruct)]),
    "amrto_mesh_info": (C.c_int, [_p, _i32p, _i32p, _i32p]),
    "amrto_set_density": (C.c_int, [_p, _p]),
    "amrto_apply": (C.c_int, [_p, _p, _p, C.c_int]),
    "amrto_project_rhs": (C.c_int, [_p, _p, _p]),
    "amrto_recover": (C.c_int, [_p, _p, _p]),
    "amrto_get_diag": (C.c_int, [_p, _p]),
    "amrto_get_block_diag": (C.c_int, [_p, _p]),
    "amrto_solve_opts_default": (None, [C.POINTER(SolveOpts)]),
    "amrto_pcg": (C.c_int, [_p, _p, _p, C.POINTER(SolveOpts), C.POINTER(SolveStats)]),
    "amrto_pcg_pass_times": (C.c_int, [_p, _p, _p, C.POINTER(SolveOpts), C.c_int32, C.POINTER(C.c_double),
                                       C.POINTER(C.c_double)]),
    "amrto_recycle_setup": (C.c_int, [_p, C.c_int32]),
    "amrto_recycle_harvest": (C.c_int, [_p, C.c_int32, C.POINTER(_p), C.POINTER(C.c_double),
                                        C.POINTER(C.c_double), _i32p]),
    "amrto_rayleigh_ritz": (C.c_int, [_p, C.POINTER(_p), C.c_int32, C.c_int32, C.POINTER(_p),
                                      C.POINTER(C.c_double), _i32p]),
    "amrto_compliance": (C.c_int, [_p, _p, _p, _p, C.POINTER(C.c_double), _p]),
    "amrto_filter": (C.c_int, [_p, C.c_int, C.c_double, _p, _p, _p]),
    "amrto_oc_update": (C.c_int, [_p, _p, _p, C.c_double, C.c_double, C.c_double, C.c_double, _p,
                                  C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "amrto_oc_update_noalloc": (C.c_int, [_p, _p, _p, C.c_double, C.c_double, C.c_double, C.c_double, _p,
                                          C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "amrto_design_difference": (C.c_int, [_p, _p, _p, _p, C.POINTER(C.c_double)]),
    "amrto_mask": (C.c_int, [_p, _p]),
    "amrto_coarse_setup": (C.c_int, [_p, C.c_int32, C.POINTER(_p), C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                     _i32p]),
    "amrto_coarse_clear": (C.c_int, [_p]),
    "amrto_coarse_gram": (C.c_int, [_p, _p, C.c_int64, _i32p]),
    "amrto_energy_combine": (C.c_int, [_p, _p, _p, C.POINTER(_p), C.c_int32, _p, C.POINTER(C.c_double)]),
    "amrto_grid_from_mesh": (C.c_int, [_p, C.c_int32, _p, _p, _p, C.c_double, _p, _p]),
    "amrto_grid_to_mesh": (C.c_int, [_p, C.c_int32, _p, C.c_double, _p]),
    "amrto_net_create": (C.c_int, [C.POINTER(_p), C.c_int, _p, C.c_int32, _i32p, C.c_int32, C.c_int32,
                                   C.c_int32, C.c_int32, C.c_int32, C.c_uint64]),
    "amrto_net_destroy": (C.c_int, [_p]),
    "amrto_net_last_error": (C.c_char_p, [_p]),
    "amrto_net_n_params": (C.c_int, [_p, C.POINTER(C.c_int64)]),
    "amrto_net_get_params": (C.c_int, [_p, _p]),
    "amrto_net_set_params": (C.c_int, [_p, _p]),
    "amrto_net_get_grads": (C.c_int, [_p, _p]),
    "amrto_net_get_adam": (C.c_int, [_p, _p, _p]),
    "amrto_net_set_adam": (C.c_int, [_p, _p, _p]),
    "amrto_net_forward": (C.c_int, [_p, _p, C.c_int32, _p]),
    "amrto_net_backward": (C.c_int, [_p, _p, _p]),
    "amrto_net_mse": (C.c_int, [_p, _p, _p, _p, C.c_int64, _p, C.POINTER(C.c_double)]),
    "amrto_net_adam": (C.c_int, [_p, C.c_float, C.c_float, C.c_float, C.c_float, C.c_int32]),
    "amrto_octree_create": (C.c_int, [C.POINTER(_p), C.POINTER(C.c_int32), C.c_int32]),
    "amrto_octree_destroy": (C.c_int, [_p]),
    "amrto_octree_n_leaves": (C.c_int32, [_p]),
    "amrto_octree_leaves": (C.c_int, [_p, _p, _p]),
    "amrto_octree_refine": (C.c_int, [_p, _p]),
    "amrto_octree_balance": (C.c_int, [_p]),
    "amrto_octree_adapt": (C.c_int, [_p, _p, C.c_double, C.c_double, _i32p]),
    "amrto_octree_adapt_result": (C.c_int, [_p, _p, _p, _p]),
    "amrto_octree_build_mesh": (C.c_int, [_p, C.c_int32, C.POINTER(Region), C.POINTER(Region), C.c_int32,
                                          C.c_int32, C.c_double, C.c_int32]),
    "amrto_octree_mesh_sizes": (C.c_int, [_p, _i32p, _i32p, _i32p, _i32p]),
    "amrto_octree_mesh_export": (C.c_int, [_p] + [_p] * 9),
    "amrto_octree_transfer_nodal": (C.c_int, [_p, _p, _p]),
    "amrto_mg_setup": (C.c_int, [_p, _p, C.POINTER(MgOpts)]),
    "amrto_mg_info": (C.c_int, [_p, _i32p, _p, _p, _p]),
    "amrto_mg_set_bounds": (C.c_int, [_p, _p]),
    "amrto_mg_get_bounds": (C.c_int, [_p, _p]),
    "amrto_mg_vcycle": (C.c_int, [_p, _p, _p]),
    "amrto_mg_level_apply": (C.c_int, [_p, C.c_int32, _p, _p]),
    "amrto_mg_level_diag": (C.c_int, [_p, C.c_int32, _p]),
    "amrto_mg_prolong": (C.c_int, [_p, C.c_int32, _p, _p]),
    "amrto_mg_restrict": (C.c_int, [_p, C.c_int32, _p, _p]),
    "amrto_mg_pcg": (C.c_int, [_p, _p, _p, C.c_double, C.c_int32, C.c_int32, C.POINTER(SolveStats)]),
    "amrto_mg_pass_times": (C.c_int, [_p, C.c_int32, _p]),
    "amrto_plane_create": (C.c_int, [C.POINTER(_p), C.c_int, _p]),
    "amrto_plane_destroy": (C.c_int, [_p]),
    "amrto_plane_last_error": (C.c_char_p, [_p]),
    "amrto_plane_set_material": (C.c_int, [_p, C.c_double, C.c_double, C.c_double, C.c_double]),
    "amrto_plane_upload_mesh": (C.c_int, [_p, C.POINTER(Mesh2DStruct)]),
    "amrto_plane_set_density": (C.c_int, [_p, _p]),
    "amrto_plane_apply": (C.c_int, [_p, _p, _p]),
    "amrto_plane_project_rhs": (C.c_int, [_p, _p, _p]),
    "amrto_plane_pcg": (C.c_int, [_p, _p, _p, C.c_double, C.c_int32, C.c_int32, C.POINTER(SolveStats)]),
    "amrto_plane_compliance": (C.c_int, [_p, _p, _p, _p, C.POINTER(C.c_double), _p]),
    "amrto_plane_filter": (C.c_int, [_p, C.c_int32, C.c_double, _p, _p, _p]),
    "amrto_plane_oc_update": (C.c_int, [_p, _p, _p, C.c_double, C.c_double, C.c_double, C.c_double, _p,
                                        C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "amrto_quadtree_create": (C.c_int, [C.POINTER(_p), C.POINTER(C.c_int32), C.c_int32]),
    "amrto_quadtree_destroy": (C.c_int, [_p]),
    "amrto_quadtree_n_leaves": (C.c_int32, [_p]),
    "amrto_quadtree_leaves": (C.c_int, [_p, _p, _p]),
    "amrto_quadtree_refine": (C.c_int, [_p, _p]),
    "amrto_quadtree_balance": (C.c_int, [_p]),
    "amrto_quadtree_adapt": (C.c_int, [_p, _p, C.c_double, C.c_double, _i32p]),
    "amrto_quadtree_adapt_result": (C.c_int, [_p, _p]),
    "amrto_quadtree_build_mesh": (C.c_int, [_p, C.c_int32, C.POINTER(Region), C.c_int32, C.c_int32, C.c_int32,
                                            C.c_double]),
    "amrto_quadtree_mesh_sizes": (C.c_int, [_p, _i32p, _i32p, _i32p, _i32p]),
    "amrto_quadtree_mesh_export": (C.c_int, [_p] + [_p] * 9),
    "amrto_quadtree_transfer_nodal": (C.c_int, [_p, _p, _p]),
}

_LIB = None


def exported_symbols():
    return sorted(_SIGS)


def load(path: str = LIB_PATH):
    """Load libamrto.so (after torch, so both share one HIP runtime)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    import torch  # noqa: F401  (maps torch's HIP runtime first)
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build() "
                           f"or python -m paper_1009_4975_amd.build")
    lib = C.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        assert t.flags["C_CONTIGUOUS"]
        return t.ctypes.data
    assert t.is_contiguous(), "device buffers must be contiguous"
    return t.data_ptr()


def _dev(t, dtype=None):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise AmrtoError(-1, "expected a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise AmrtoError(-1, f"expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise AmrtoError(-1, "device buffers must be contiguous")
    return t.data_ptr()


def _need(n, **bufs):
    """Raise EINVAL unless every given buffer (None skipped) holds exactly n
    values: the C ABI takes bare pointers, so a short or stale buffer would be
    read or written out of bounds on the device."""
    for name, t in bufs.items():
        if t is None:
            continue
        have = t.numel() if hasattr(t, "numel") else int(np.size(t))
        if have != n:
            raise AmrtoError(-1, f"{name} has {have} values, {n} expected")


# ---------------------------------------------------------------------- mesh
@dataclass
class MeshArrays:
    """Host arrays of a mesh as produced by the octree (``Octree.mesh``)."""
    dims: tuple
    max_level: int
    node_xyz: np.ndarray          # (nn, 3) int32
    elem_nodes: np.ndarray        # (ne, 8) int32
    elem_level: np.ndarray        # (ne,) int8
    hang_node: np.ndarray         # (nh,) int32
    hang_ptr: np.ndarray          # (nh+1,) int32
    hang_master: np.ndarray       # int32
    hang_w: np.ndarray            # float64
    dof_fixed: np.ndarray         # (3 nn,) uint8
    f_load: np.ndarray            # (3 nn,) float64
    uniform: bool = False

    @property
    def n_nodes(self):
        return len(self.node_xyz)

    @property
    def n_elems(self):
        return len(self.elem_level)

    def struct(self):
        keep = []

        def arr(a, dt):
            a = np.ascontiguousarray(a, dtype=dt)
            keep.append(a)
            return a.ctypes.data

        m = MeshStruct()
        m.n_nodes = self.n_nodes
        m.n_elems = self.n_elems
        m.dims[:] = list(self.dims)
        m.max_level = self.max_level
        m.node_xyz = None if self.uniform else arr(self.node_xyz, np.int32)
        m.elem_nodes = None if self.uniform else arr(self.elem_nodes, np.int32)
        m.elem_level = arr(self.elem_level, np.int8)
        m.n_hang = 0 if self.uniform else len(self.hang_node)
        m.hang_node = arr(self.hang_node, np.int32)
        m.hang_ptr = arr(self.hang_ptr, np.int32)
        m.hang_master = arr(self.hang_master, np.int32)
        m.hang_w = arr(self.hang_w, np.float64)
        m.dof_fixed = arr(self.dof_fixed, np.uint8)
        return m, keep


def _region(where: dict) -> Region:
    r = Region()
    axes = {"x": 0, "y": 1, "z": 2}
    for k, v in where.items():
        r.has[axes[k]] = 1
        r.at[axes[k]] = int(v)
    return r


class Octree:
    """Host octree (refine, closure, adapt, mesh build) in libamrto.so."""

    def __init__(self, base, max_level):
        self.lib = load()
        self.h = _p()
        b = (C.c_int32 * 3)(*base)
        self._chk(self.lib.amrto_octree_create(C.byref(self.h), b, int(max_level)))
        self.base = tuple(base)
        self.max_level = int(max_level)
        self.dims = tuple(int(x) << self.max_level for x in base)

    def _chk(self, rc):
        if rc < 0:
            raise AmrtoError(rc, "octree call failed")
        return rc

    def __del__(self):
        try:
            if getattr(self, "h", None) and self.h.value:
                self.lib.amrto_octree_destroy(self.h)
                self.h = _p()
        except Exception:  # interpreter shutdown: ctypes may already be gone
            pass

    def leaves(self):
        n = self.lib.amrto_octree_n_leaves(self.h)
        lv = np.zeros(n, np.int8)
        an = np.zeros((n, 3), np.int32)
        self._chk(self.lib.amrto_octree_leaves(self.h, lv.ctypes.data, an.ctypes.data))
        return lv.astype(np.int64), an.astype(np.int64)

    def refine(self, marks):
        m = np.ascontiguousarray(np.asarray(marks, dtype=np.uint8))
        assert len(m) == self.lib.amrto_octree_n_leaves(self.h)
        self._chk(self.lib.amrto_octree_refine(self.h, m.ctypes.data))

    def balance(self):
        self._chk(self.lib.amrto_octree_balance(self.h))

    def adapt(self, rho, rho_s=0.5, r_amr=1.5):
        r = np.ascontiguousarray(rho, dtype=np.float64)
        assert len(r) == self.lib.amrto_octree_n_leaves(self.h)
        n = C.c_int32()
        self._chk(self.lib.amrto_octree_adapt(self.h, r.ctypes.data, rho_s, r_amr, C.byref(n)))
        out = np.zeros(n.value)
        self._chk(self.lib.amrto_octree_adapt_result(self.h, out.ctypes.data, None, None))
        return out

    def build_mesh(self, fixed, load, lexicographic=False) -> MeshArrays:
        regs = (Region * max(1, len(fixed)))(*[_region(w) for w in fixed])
        lr = _region(load["where"])
        kind = 0 if load["kind"] == "line" else 1
        self._chk(self.lib.amrto_octree_build_mesh(self.h, len(fixed), regs, C.byref(lr), kind,
                                                   int(load["comp"]), float(load["total"]),
                                                   1 if lexicographic else 0))
        nn, ne, nh, nhe = (C.c_int32() for _ in range(4))
        self._chk(self.lib.amrto_octree_mesh_sizes(self.h, C.byref(nn), C.byref(ne), C.byref(nh), C.byref(nhe)))
        nn, ne, nh, nhe = nn.value, ne.value, nh.value, nhe.value
        xyz = np.zeros((nn, 3), np.int32)
        en = np.zeros((ne, 8), np.int32)
        lv = np.zeros(ne, np.int8)
        hn = np.zeros(nh, np.int32)
        hp = np.zeros(nh + 1, np.int32)
        hm = np.zeros(nhe, np.int32)
        hw = np.zeros(nhe, np.float64)
        fx = np.zeros(3 * nn, np.uint8)
        fl = np.zeros(3 * nn, np.float64)
        self._chk(self.lib.amrto_octree_mesh_export(self.h, *[a.ctypes.data for a in (xyz, en, lv, hn, hp, hm, hw,
                                                                                          fx, fl)]))
        return MeshArrays(self.dims, self.max_level, xyz, en, lv, hn, hp, hm, hw, fx, fl,
                          uniform=False)

    def transfer_nodal(self, u_old: np.ndarray, n_new_nodes: int) -> np.ndarray:
        u_old = np.ascontiguousarray(u_old, dtype=np.float64)
        out = np.zeros(3 * n_new_nodes)
        self._chk(self.lib.amrto_octree_transfer_nodal(self.h, u_old.ctypes.data, out.ctypes.data))
        return out


def uniform_mesh(dims, fixed, load, tree=None) -> MeshArrays:
    """A uniform brick (implicit connectivity on the device): the octree with
    one level and lexicographic node numbering supplies supports and loads
    (pass ``tree = Octree(dims, 0)`` to keep it, e.g. for the multigrid)."""
    t = Octree(dims, 0) if tree is None else tree
    m = t.build_mesh(fixed, load, lexicographic=True)
    m.uniform = True
    return m


# ---------------------------------------------------------------------- context
class Context:
    """A device context: mesh, coefficients, preconditioner and workspace."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.lib = load()
        self.torch = torch
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        self.h = _p()
        rc = self.lib.amrto_create(C.byref(self.h), int(device), _p(stream.cuda_stream))
        if rc != 0:
            raise AmrtoError(rc, "amrto_create failed")
        self.device = device
        self.mesh: Optional[MeshArrays] = None

    def __del__(self):
        try:
            if getattr(self, "h", None) and self.h.value:
                self.lib.amrto_destroy(self.h)
                self.h = _p()
        except Exception:  # interpreter shutdown: ctypes may already be gone
            pass

    def _chk(self, rc, allow_not_converged=False):
        if rc < 0 or (rc > 0 and not allow_not_converged):
            raise AmrtoError(rc, self.lib.amrto_last_error(self.h).decode())
        return rc

    def set_material(self, E0=1.0, Emin=1e-9, nu=0.3, p=3.0):
        self._chk(self.lib.amrto_set_material(self.h, E0, Emin, nu, p))

    def set_deterministic(self, on=True):
        self._chk(self.lib.amrto_set_deterministic(self.h, 1 if on else 0))

    def upload_mesh(self, mesh: MeshArrays):
        s, keep = mesh.struct()
        self.mesh = None
        self._chk(self.lib.amrto_upload_mesh(self.h, C.byref(s)))
        del keep
        self.mesh = mesh

    @property
    def _n3(self):
        """DOF-vector length of the uploaded mesh (None before an upload: the
        library then answers ESTATE itself)."""
        return None if self.mesh is None else 3 * self.mesh.n_nodes

    @property
    def _ne(self):
        return None if self.mesh is None else self.mesh.n_elems

    def _dofs(self, **bufs):
        if self.mesh is not None:
            _need(self._n3, **bufs)

    def _elems(self, **bufs):
        if self.mesh is not None:
            _need(self._ne, **bufs)

    def info(self):
        a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
        self._chk(self.lib.amrto_mesh_info(self.h, C.byref(a), C.byref(b), C.byref(c)))
        return dict(n_nodes=a.value, n_elems=b.value, n_chunks=c.value)

    def set_density(self, rho):
        self._elems(rho=rho)
        self._chk(self.lib.amrto_set_density(self.h, _dev(rho, self.torch.float64)))

    def apply(self, x, y, prec=FP64):
        dt = self.torch.float64 if prec == FP64 else self.torch.float32
        self._dofs(x=x, y=y)
        self._chk(self.lib.amrto_apply(self.h, _dev(x, dt), _dev(y, dt), int(prec)))

    def project_rhs(self, f, b):
        self._dofs(f=f, b=b)
        self._chk(self.lib.amrto_project_rhs(self.h, _dev(f, self.torch.float64), _dev(b, self.torch.float64)))

    def recover(self, ut, u):
        self._dofs(ut=ut, u=u)
        self._chk(self.lib.amrto_recover(self.h, _dev(ut, self.torch.float64), _dev(u, self.torch.float64)))

    def diag(self, out):
        self._dofs(out=out)
        self._chk(self.lib.amrto_get_diag(self.h, _dev(out, self.torch.float64)))

    def block_diag(self, out):
        """3x3 node blocks of A~ into out (9 n_nodes float64, row-major per node)."""
        if self.mesh is not None:
            _need(9 * self.mesh.n_nodes, out=out)
        self._chk(self.lib.amrto_get_block_diag(self.h, _dev(out, self.torch.float64)))

    def pcg(self, b, u, rtol=1e-8, max_it=20000, inner_prec=FP64, inner_rtol=0.1, check_every=16,
            use_coarse=True, fallback_fp64=True, single_reduction=False, precond=JACOBI,
            allow_not_converged=False, record=False):
        self._dofs(b=b, u=u)
        o = SolveOpts()
        self.lib.amrto_solve_opts_default(C.byref(o))
        o.rtol, o.max_it, o.inner_prec, o.inner_rtol = rtol, max_it, inner_prec, inner_rtol
        o.precond = int(precond)
        o.check_every, o.use_coarse = check_every, int(bool(use_coarse))
        o.fallback_fp64 = int(bool(fallback_fp64))
        o.single_reduction = int(bool(single_reduction))
        o.record = int(bool(record))
        st = SolveStats()
        rc = self.lib.amrto_pcg(self.h, _dev(b, self.torch.float64), _dev(u, self.torch.float64), C.byref(o),
                                C.byref(st))
        self._chk(rc, allow_not_converged=allow_not_converged)
        return dict(iters=st.iters, outer=st.outer, rel_res=st.rel_res, ms=st.ms, status=STATUS[rc],
                    fell_back=bool(st.fell_back))

    def recycle_setup(self, m):
        self._chk(self.lib.amrto_recycle_setup(self.h, int(m)))

    def recycle_harvest(self, outs):
        """Ritz vectors of the last recorded solve into the FP64 DOF vectors
        `outs`; returns (theta, residual norms, Lanczos steps used)."""
        k = len(outs)
        self._dofs(**{f"outs[{i}]": o for i, o in enumerate(outs)})
        arr = (_p * k)(*[_dev(o, self.torch.float64) for o in outs])
        th, rs, m = (C.c_double * k)(), (C.c_double * k)(), C.c_int32()
        self._chk(self.lib.amrto_recycle_harvest(self.h, k, arr, th, rs, C.byref(m)))
        return list(th), list(rs), m.value

    def rayleigh_ritz(self, vecs, outs):
        """The len(outs) smallest Rayleigh-Ritz pairs of (A~, diag A~) on
        span(vecs); returns (theta, rank kept)."""
        n, k = len(vecs), len(outs)
        self._dofs(**{f"vecs[{i}]": v for i, v in enumerate(vecs)}, **{f"outs[{i}]": o for i, o in enumerate(outs)})
        sa = (_p * n)(*[_dev(v, self.torch.float64) for v in vecs])
        wa = (_p * k)(*[_dev(o, self.torch.float64) for o in outs])
        th, rank = (C.c_double * k)(), C.c_int32()
        self._chk(self.lib.amrto_rayleigh_ritz(self.h, sa, n, k, wa, th, C.byref(rank)))
        return list(th), rank.value

    def pcg_pass_times(self, b, u, reps=200, inner_prec=FP64, precond=JACOBI, use_coarse=True):
        """Mean device time (us) of one launch of the solver variant's operator
        pass and of its update side (amrto_pcg_pass_times)."""
        self._dofs(b=b, u=u)
        o = SolveOpts()
        self.lib.amrto_solve_opts_default(C.byref(o))
        o.inner_prec, o.precond, o.use_coarse = inner_prec, int(precond), int(bool(use_coarse))
        op, up = C.c_double(), C.c_double()
        self._chk(self.lib.amrto_pcg_pass_times(self.h, _dev(b, self.torch.float64), _dev(u, self.torch.float64),
                                                C.byref(o), int(reps), C.byref(op), C.byref(up)))
        return op.value, up.value

    # ------------------------------------------------------------ multigrid
    def mg_setup(self, tree, degree=2, ratio=10.0, power_its=20, hi_factor=1.1, coarse_dofs=200, first=1,
                 coarse_degree=0, blocks0=False):
        """Multigrid hierarchy of the uploaded mesh from the host tree it was built from."""
        o = MgOpts(int(degree), float(ratio), int(power_its), float(hi_factor), int(coarse_dofs), int(first),
                   int(coarse_degree), int(bool(blocks0)))
        self._mg_dofs = None
        self._chk(self.lib.amrto_mg_setup(self.h, tree.h, C.byref(o)))
        self._mg_dofs = self.mg_info()["dofs"]

    def mg_info(self):
        n = C.c_int32()
        dofs = np.zeros(16, np.int32)
        dense = np.zeros(16, np.int32)
        blocks = np.zeros(16, np.int64)
        self._chk(self.lib.amrto_mg_info(self.h, C.byref(n), dofs.ctypes.data, dense.ctypes.data,
                                         blocks.ctypes.data))
        return dict(levels=n.value, dofs=dofs[:n.value].tolist(), dense=dense[:n.value].tolist(),
                    blocks=blocks[:n.value].tolist())

    def _mg_level(self, k):
        dofs = getattr(self, "_mg_dofs", None)
        if dofs is None:
            raise AmrtoError(-5, "no multigrid hierarchy (mg_setup)")
        if not 1 <= k < len(dofs):
            raise AmrtoError(-1, f"level {k} out of range 1..{len(dofs) - 1}")
        return dofs

    def mg_set_bounds(self, lam=None):
        if lam is None:
            self._chk(self.lib.amrto_mg_set_bounds(self.h, None))
            return
        dofs = getattr(self, "_mg_dofs", None) or []
        a = np.ascontiguousarray(lam, dtype=np.float64)
        if len(a) != max(0, len(dofs) - 1):
            raise AmrtoError(-1, f"{len(a)} bounds given, {max(0, len(dofs) - 1)} smoothed levels")
        self._chk(self.lib.amrto_mg_set_bounds(self.h, a.ctypes.data))

    def mg_get_bounds(self):
        dofs = getattr(self, "_mg_dofs", None) or []
        out = np.zeros(max(1, len(dofs) - 1))
        self._chk(self.lib.amrto_mg_get_bounds(self.h, out.ctypes.data))
        return out[:max(0, len(dofs) - 1)]

    def mg_vcycle(self, r, z):
        self._dofs(r=r, z=z)
        self._chk(self.lib.amrto_mg_vcycle(self.h, _dev(r, self.torch.float64), _dev(z, self.torch.float64)))

    def mg_level_apply(self, k, x, y):
        dofs = self._mg_level(k)
        _need(dofs[k], x=x, y=y)
        self._chk(self.lib.amrto_mg_level_apply(self.h, int(k), _dev(x, self.torch.float64),
                                                _dev(y, self.torch.float64)))

    def mg_level_diag(self, k, out):
        dofs = self._mg_level(k)
        _need(dofs[k], out=out)
        self._chk(self.lib.amrto_mg_level_diag(self.h, int(k), _dev(out, self.torch.float64)))

    def mg_prolong(self, k, xc, xf):
        dofs = self._mg_level(k)
        _need(dofs[k], xc=xc)
        _need(dofs[k - 1], xf=xf)
        self._chk(self.lib.amrto_mg_prolong(self.h, int(k), _dev(xc, self.torch.float64),
                                            _dev(xf, self.torch.float64)))

    def mg_restrict(self, k, rf, rc):
        dofs = self._mg_level(k)
        _need(dofs[k - 1], rf=rf)
        _need(dofs[k], rc=rc)
        self._chk(self.lib.amrto_mg_restrict(self.h, int(k), _dev(rf, self.torch.float64),
                                             _dev(rc, self.torch.float64)))

    def mg_pass_times(self, reps=100):
        """Mean us of one smoothing pass per smoothed level (level 0 first)."""
        dofs = getattr(self, "_mg_dofs", None) or []
        out = np.zeros(max(1, len(dofs) - 1))
        self._chk(self.lib.amrto_mg_pass_times(self.h, int(reps), out.ctypes.data))
        return out[:max(0, len(dofs) - 1)].tolist()

    def mg_pcg(self, b, u, rtol=1e-8, max_it=5000, check_every=2):
        self._dofs(b=b, u=u)
        st = SolveStats()
        rc = self.lib.amrto_mg_pcg(self.h, _dev(b, self.torch.float64), _dev(u, self.torch.float64), float(rtol),
                                   int(max_it), int(check_every), C.byref(st))
        self._chk(rc, allow_not_converged=True)
        return dict(status=STATUS.get(rc, rc), iters=st.iters, outer=st.outer, rel_res=st.rel_res, ms=st.ms,
                    fell_back=0)

    def compliance(self, u, f, rho=None, dc=None):
        self._dofs(u=u, f=f)
        self._elems(rho=rho, dc=dc)
        c = C.c_double()
        self._chk(self.lib.amrto_compliance(self.h, _dev(u, self.torch.float64), _dev(f, self.torch.float64),
                                            None if rho is None else _dev(rho, self.torch.float64),
                                            C.byref(c), None if dc is None else _dev(dc, self.torch.float64)))
        return c.value

    def sensitivity(self, u, rho, dc):
        self._dofs(u=u)
        self._elems(rho=rho, dc=dc)
        self._chk(self.lib.amrto_compliance(self.h, _dev(u, self.torch.float64), None,
                                            _dev(rho, self.torch.float64), None, _dev(dc, self.torch.float64)))

    def filter(self, mode, rmin, inp, out, rho=None):
        self._elems(inp=inp, out=out, rho=rho)
        self._chk(self.lib.amrto_filter(self.h, int(mode), float(rmin), _dev(inp, self.torch.float64),
                                        None if rho is None else _dev(rho, self.torch.float64),
                                        _dev(out, self.torch.float64)))

    def oc_update(self, rho, dc, rho_new, volfrac, move=0.2, eta=0.5, rho_min=1e-3):
        self._elems(rho=rho, dc=dc, rho_new=rho_new)
        ch, lam = C.c_double(), C.c_double()
        self._chk(self.lib.amrto_oc_update(self.h, _dev(rho, self.torch.float64), _dev(dc, self.torch.float64),
                                           volfrac, move, eta, rho_min, _dev(rho_new, self.torch.float64),
                                           C.byref(ch), C.byref(lam)))
        return ch.value, lam.value

    def oc_update_noalloc(self, rho, dc, rho_new, volfrac, move=0.2, eta=0.5, rho_min=1e-3):
        """amrto_oc_update on the library's per-GPU static scratch (no workspace of the context)."""
        self._elems(rho=rho, dc=dc, rho_new=rho_new)
        ch, lam = C.c_double(), C.c_double()
        self._chk(self.lib.amrto_oc_update_noalloc(self.h, _dev(rho, self.torch.float64),
                                                   _dev(dc, self.torch.float64), volfrac, move, eta, rho_min,
                                                   _dev(rho_new, self.torch.float64), C.byref(ch), C.byref(lam)))
        return ch.value, lam.value

    def design_difference(self, rho, other, rho_other):
        """Eq. (10) between this context's design rho and other's rho_other."""
        self._elems(rho=rho)
        other._elems(rho_other=rho_other)
        d = C.c_double()
        self._chk(self.lib.amrto_design_difference(self.h, _dev(rho, self.torch.float64), other.h,
                                                   _dev(rho_other, self.torch.float64), C.byref(d)))
        return d.value

    def mask(self, x):
        self._dofs(x=x)
        self._chk(self.lib.amrto_mask(self.h, _dev(x, self.torch.float64)))

    def coarse_setup(self, fields, rx, ry, rz, affine=False):
        """fields: sequence of float64 device vectors (3n); returns the rank kept."""
        n = len(fields)
        self._dofs(**{f"fields[{i}]": f for i, f in enumerate(fields)})
        arr = (_p * max(n, 1))(*[_dev(f, self.torch.float64) for f in fields])
        kept = C.c_int32()
        self._chk(self.lib.amrto_coarse_setup(self.h, int(bool(affine)), arr, n, int(rx), int(ry), int(rz),
                                              C.byref(kept)))
        return kept.value

    def coarse_clear(self):
        self._chk(self.lib.amrto_coarse_clear(self.h))

    def coarse_gram(self):
        """The Gram matrix Z^T A~ Z of the current coarse space (k x k numpy array)."""
        k = C.c_int32()
        cap = 384 * 384
        buf = np.empty(cap, np.float64)
        self._chk(self.lib.amrto_coarse_gram(self.h, buf.ctypes.data_as(_p), cap, C.byref(k)))
        return buf[: k.value * k.value].reshape(k.value, k.value).copy()

    def energy_combine(self, b, vecs, x0, base=None):
        n = len(vecs)
        self._dofs(b=b, x0=x0, base=base, **{f"vecs[{i}]": v for i, v in enumerate(vecs)})
        f64 = self.torch.float64
        arr = (_p * n)(*[_dev(v, f64) for v in vecs])
        coef = (C.c_double * n)()
        self._chk(self.lib.amrto_energy_combine(self.h, _dev(b, f64), None if base is None else _dev(base, f64),
                                                arr, n, _dev(x0, f64), coef))
        return list(coef)

    def _grid_nodes(self, cell):
        """Node count of the regular grid with nodes every `cell` lattice units
        (None when there is no mesh or the cell does not divide the extents:
        the library rejects those itself)."""
        if self.mesh is None or cell <= 0 or any(int(d) % int(cell) for d in self.mesh.dims):
            return None
        gx, gy, gz = (int(d) // int(cell) for d in self.mesh.dims)
        return (gx + 1) * (gy + 1) * (gz + 1)

    def grid_from_mesh(self, cell, rho=None, u=None, rho_grid=None, u_grid=None, u_scale=1.0, u_ref=None):
        f64, f32 = self.torch.float64, self.torch.float32
        self._dofs(u=u, u_ref=u_ref)
        self._elems(rho=rho)
        g = self._grid_nodes(cell)
        if g is not None:
            _need(g, rho_grid=rho_grid)
            _need(3 * g, u_grid=u_grid)
        self._chk(self.lib.amrto_grid_from_mesh(
            self.h, int(cell), None if rho is None else _dev(rho, f64), None if u is None else _dev(u, f64),
            None if u_ref is None else _dev(u_ref, f64), float(u_scale),
            None if rho_grid is None else _dev(rho_grid, f32), None if u_grid is None else _dev(u_grid, f32)))

    def grid_to_mesh(self, cell, u_grid, u, scale=1.0):
        self._dofs(u=u)
        g = self._grid_nodes(cell)
        if g is not None:
            _need(3 * g, u_grid=u_grid)
        self._chk(self.lib.amrto_grid_to_mesh(self.h, int(cell), _dev(u_grid, self.torch.float32), float(scale),
                                              _dev(u, self.torch.float64)))


class Net:
    """3x3x3 convolution stack on a regular grid, trained by the library's kernels."""

    def __init__(self, channels, grid, max_batch=1, seed=0, skip_from=-1, device=0, stream=None):
        self.lib = load()
        import torch
        self.torch = torch
        self.channels = [int(c) for c in channels]
        self.grid = tuple(int(g) for g in grid)  # (gx, gy, gz)
        ch = (C.c_int32 * len(self.channels))(*self.channels)
        h = _p()
        st = stream if stream is not None else torch.cuda.current_stream(device).cuda_stream
        rc = self.lib.amrto_net_create(C.byref(h), int(device), st, len(self.channels) - 1, ch, int(skip_from),
                                       *self.grid, int(max_batch), int(seed))
        if rc != 0:
            raise AmrtoError(rc, "amrto_net_create failed")
        self.h = h

    def __del__(self):
        try:
            if getattr(self, "h", None):
                self.lib.amrto_net_destroy(self.h)
                self.h = None
        except Exception:  # interpreter shutdown: ctypes may already be gone
            pass

    def _chk(self, rc):
        if rc != 0:
            raise AmrtoError(rc, self.lib.amrto_net_last_error(self.h).decode())

    def n_params(self):
        n = C.c_int64()
        self._chk(self.lib.amrto_net_n_params(self.h, C.byref(n)))
        return n.value

    def get_params(self):
        out = np.empty(self.n_params(), np.float32)
        self._chk(self.lib.amrto_net_get_params(self.h, out.ctypes.data))
        return out

    def set_params(self, flat):
        a = np.ascontiguousarray(flat, dtype=np.float32)
        assert a.size == self.n_params()
        self._chk(self.lib.amrto_net_set_params(self.h, a.ctypes.data))

    def get_grads(self):
        out = np.empty(self.n_params(), np.float32)
        self._chk(self.lib.amrto_net_get_grads(self.h, out.ctypes.data))
        return out

    def get_adam(self):
        """Adam moments (m, v) as host arrays."""
        m = np.empty(self.n_params(), np.float32)
        v = np.empty_like(m)
        self._chk(self.lib.amrto_net_get_adam(self.h, m.ctypes.data, v.ctypes.data))
        return m, v

    def set_adam(self, m, v):
        m = np.ascontiguousarray(m, dtype=np.float32)
        v = np.ascontiguousarray(v, dtype=np.float32)
        assert m.size == v.size == self.n_params()
        self._chk(self.lib.amrto_net_set_adam(self.h, m.ctypes.data, v.ctypes.data))

    def _act(self, batch, ch):
        gx, gy, gz = self.grid
        return batch * ch * gx * gy * gz

    def forward(self, x, out):
        batch = int(x.shape[0]) if x.dim() > 0 else 0
        _need(self._act(batch, self.channels[0]), x=x)
        _need(self._act(batch, self.channels[-1]), out=out)
        self._batch = batch
        self._chk(self.lib.amrto_net_forward(self.h, _dev(x, self.torch.float32), int(x.shape[0]),
                                             _dev(out, self.torch.float32)))

    def backward(self, dout, din=None):
        batch = getattr(self, "_batch", None)
        if batch is not None:
            _need(self._act(batch, self.channels[-1]), dout=dout)
            _need(self._act(batch, self.channels[0]), din=din)
        self._chk(self.lib.amrto_net_backward(self.h, _dev(dout, self.torch.float32),
                                              None if din is None else _dev(din, self.torch.float32)))

    def mse(self, pred, target, dpred, mask=None):
        _need(pred.numel(), target=target, dpred=dpred, mask=mask)
        loss = C.c_double()
        self._chk(self.lib.amrto_net_mse(self.h, _dev(pred, self.torch.float32), _dev(target, self.torch.float32),
                                         None if mask is None else _dev(mask, self.torch.uint8), int(pred.numel()),
                                         _dev(dpred, self.torch.float32), C.byref(loss)))
        return loss.value

    def adam(self, lr, t, beta1=0.9, beta2=0.999, eps=1e-8):
        self._chk(self.lib.amrto_net_adam(self.h, lr, beta1, beta2, eps, int(t)))


# ---------------------------------------------------------------------- 2-D variant
@dataclass
class Mesh2DArrays:
    """Host arrays of a quadtree mesh (``Quadtree.build_mesh``)."""
    dims: tuple
    max_level: int
    node_xy: np.ndarray           # (nn, 2) int32, x fastest
    elem_nodes: np.ndarray        # (ne, 4) int32, local a = i + 2 j
    elem_level: np.ndarray        # (ne,) int8
    hang_node: np.ndarray
    hang_ptr: np.ndarray
    hang_master: np.ndarray
    hang_w: np.ndarray
    dof_fixed: np.ndarray         # (2 nn,) uint8
    f_load: np.ndarray            # (2 nn,) float64

    @property
    def n_nodes(self):
        return len(self.node_xy)

    @property
    def n_elems(self):
        return len(self.elem_level)

    def struct(self):
        keep = []

        def arr(a, dt):
            a = np.ascontiguousarray(a, dtype=dt)
            keep.append(a)
            return a.ctypes.data

        m = Mesh2DStruct()
        m.n_nodes, m.n_elems = self.n_nodes, self.n_elems
        m.dims[:] = list(self.dims)
        m.max_level = self.max_level
        m.node_xy = arr(self.node_xy, np.int32)
        m.elem_nodes = arr(self.elem_nodes, np.int32)
        m.elem_level = arr(self.elem_level, np.int8)
        m.n_hang = len(self.hang_node)
        m.hang_node = arr(self.hang_node, np.int32)
        m.hang_ptr = arr(self.hang_ptr, np.int32)
        m.hang_master = arr(self.hang_master, np.int32)
        m.hang_w = arr(self.hang_w, np.float64)
        m.dof_fixed = arr(self.dof_fixed, np.uint8)
        return m, keep


class Quadtree:
    """Host quadtree of the 2-D variant (refine, closure, adapt, mesh build)."""

    def __init__(self, base, max_level):
        self.lib = load()
        self.h = _p()
        b = (C.c_int32 * 2)(*base)
        self._chk(self.lib.amrto_quadtree_create(C.byref(self.h), b, int(max_level)))
        self.base = tuple(base)
        self.max_level = int(max_level)
        self.dims = tuple(int(x) << self.max_level for x in base)

    def _chk(self, rc):
        if rc < 0:
            raise AmrtoError(rc, "quadtree call failed")
        return rc

    def __del__(self):
        try:
            if getattr(self, "h", None) and self.h.value:
                self.lib.amrto_quadtree_destroy(self.h)
                self.h = _p()
        except Exception:  # interpreter shutdown: ctypes may already be gone
            pass

    @property
    def n_leaves(self):
        return self.lib.amrto_quadtree_n_leaves(self.h)

    def leaves(self):
        n = self.n_leaves
        lv = np.zeros(n, np.int8)
        an = np.zeros((n, 2), np.int32)
        self._chk(self.lib.amrto_quadtree_leaves(self.h, lv.ctypes.data, an.ctypes.data))
        return lv.astype(np.int64), an.astype(np.int64)

    def refine(self, marks):
        m = np.ascontiguousarray(marks, dtype=np.uint8)
        if len(m) != self.n_leaves:
            raise AmrtoError(-1, f"marks has {len(m)} values, {self.n_leaves} expected")
        self._chk(self.lib.amrto_quadtree_refine(self.h, m.ctypes.data))

    def balance(self):
        self._chk(self.lib.amrto_quadtree_balance(self.h))

    def adapt(self, rho, rho_s=0.5, r_amr=1.5):
        r = np.ascontiguousarray(rho, dtype=np.float64)
        if len(r) != self.n_leaves:
            raise AmrtoError(-1, f"rho has {len(r)} values, {self.n_leaves} expected")
        n = C.c_int32()
        self._chk(self.lib.amrto_quadtree_adapt(self.h, r.ctypes.data, rho_s, r_amr, C.byref(n)))
        out = np.zeros(n.value)
        self._chk(self.lib.amrto_quadtree_adapt_result(self.h, out.ctypes.data))
        return out

    def build_mesh(self, fixed, load) -> Mesh2DArrays:
        """fixed: list of {"x": v} / {"y": v} / {"x": v, "y": w}; load:
        {"at": (x, y), "comp": c, "total": F}."""
        regs = (Region * max(1, len(fixed)))(*[_region(w) for w in fixed])
        x, y = load["at"]
        self._chk(self.lib.amrto_quadtree_build_mesh(self.h, len(fixed), regs, int(x), int(y), int(load["comp"]),
                                                     float(load["total"])))
        nn, ne, nh, nhe = (C.c_int32() for _ in range(4))
        self._chk(self.lib.amrto_quadtree_mesh_sizes(self.h, C.byref(nn), C.byref(ne), C.byref(nh), C.byref(nhe)))
        nn, ne, nh, nhe = nn.value, ne.value, nh.value, nhe.value
        xy = np.zeros((nn, 2), np.int32)
        en = np.zeros((ne, 4), np.int32)
        lv = np.zeros(ne, np.int8)
        hn = np.zeros(nh, np.int32)
        hp = np.zeros(nh + 1, np.int32)
        hm = np.zeros(nhe, np.int32)
        hw = np.zeros(nhe, np.float64)
        fx = np.zeros(2 * nn, np.uint8)
        fl = np.zeros(2 * nn, np.float64)
        self._chk(self.lib.amrto_quadtree_mesh_export(self.h, *[a.ctypes.data for a in (xy, en, lv, hn, hp, hm, hw,
                                                                                            fx, fl)]))
        return Mesh2DArrays(self.dims, self.max_level, xy, en, lv, hn, hp, hm, hw, fx, fl)

    def transfer_nodal(self, u_old: np.ndarray, n_new_nodes: int) -> np.ndarray:
        u_old = np.ascontiguousarray(u_old, dtype=np.float64)
        out = np.zeros(2 * n_new_nodes)
        self._chk(self.lib.amrto_quadtree_transfer_nodal(self.h, u_old.ctypes.data, out.ctypes.data))
        return out


class PlaneContext:
    """Device context of the 2-D variant (amrto_plane_*)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.lib = load()
        self.torch = torch
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        self.h = _p()
        rc = self.lib.amrto_plane_create(C.byref(self.h), int(device), _p(stream.cuda_stream))
        if rc != 0:
            raise AmrtoError(rc, "amrto_plane_create failed")
        self.mesh: Optional[Mesh2DArrays] = None

    def __del__(self):
        try:
            if getattr(self, "h", None) and self.h.value:
                self.lib.amrto_plane_destroy(self.h)
                self.h = _p()
        except Exception:  # interpreter shutdown: ctypes may already be gone
            pass

    def _chk(self, rc, allow_not_converged=False):
        if rc < 0 or (rc > 0 and not allow_not_converged):
            raise AmrtoError(rc, self.lib.amrto_plane_last_error(self.h).decode())
        return rc

    def _dofs(self, **bufs):
        if self.mesh is not None:
            _need(2 * self.mesh.n_nodes, **bufs)

    def _elems(self, **bufs):
        if self.mesh is not None:
            _need(self.mesh.n_elems, **bufs)

    def set_material(self, E0=1.0, Emin=1e-9, nu=0.3, p=3.0):
        self._chk(self.lib.amrto_plane_set_material(self.h, E0, Emin, nu, p))

    def upload_mesh(self, mesh: Mesh2DArrays):
        s, keep = mesh.struct()
        self.mesh = None
        self._chk(self.lib.amrto_plane_upload_mesh(self.h, C.byref(s)))
        del keep
        self.mesh = mesh

    def set_density(self, rho):
        self._elems(rho=rho)
        self._chk(self.lib.amrto_plane_set_density(self.h, _dev(rho, self.torch.float64)))

    def apply(self, x, y):
        self._dofs(x=x, y=y)
        self._chk(self.lib.amrto_plane_apply(self.h, _dev(x, self.torch.float64), _dev(y, self.torch.float64)))

    def project_rhs(self, f, b):
        self._dofs(f=f, b=b)
        self._chk(self.lib.amrto_plane_project_rhs(self.h, _dev(f, self.torch.float64),
                                                   _dev(b, self.torch.float64)))

    def pcg(self, b, u, rtol=1e-8, max_it=20000, check_every=16):
        self._dofs(b=b, u=u)
        st = SolveStats()
        rc = self.lib.amrto_plane_pcg(self.h, _dev(b, self.torch.float64), _dev(u, self.torch.float64),
                                      float(rtol), int(max_it), int(check_every), C.byref(st))
        self._chk(rc, allow_not_converged=True)
        return dict(status=STATUS.get(rc, rc), iters=st.iters, outer=st.outer, rel_res=st.rel_res, ms=st.ms)

    def compliance(self, u, f=None, rho=None, dc=None):
        self._dofs(u=u, f=f)
        self._elems(rho=rho, dc=dc)
        c = C.c_double()
        f64 = self.torch.float64
        self._chk(self.lib.amrto_plane_compliance(
            self.h, _dev(u, f64), None if f is None else _dev(f, f64), None if rho is None else _dev(rho, f64),
            C.byref(c) if f is not None else None, None if dc is None else _dev(dc, f64)))
        return c.value if f is not None else None

    def filter(self, mode, rmin, x, out, rho=None):
        self._elems(x=x, out=out, rho=rho)
        f64 = self.torch.float64
        self._chk(self.lib.amrto_plane_filter(self.h, int(mode), float(rmin), _dev(x, f64),
                                              None if rho is None else _dev(rho, f64), _dev(out, f64)))

    def oc_update(self, rho, dc, rho_new, volfrac, move=0.2, eta=0.5, rho_min=1e-3):
        self._elems(rho=rho, dc=dc, rho_new=rho_new)
        ch, lam = C.c_double(), C.c_double()
        f64 = self.torch.float64
        self._chk(self.lib.amrto_plane_oc_update(self.h, _dev(rho, f64), _dev(dc, f64), float(volfrac),
                                                 float(move), float(eta), float(rho_min), _dev(rho_new, f64),
                                                 C.byref(ch), C.byref(lam)))
        return ch.value, lam.value
