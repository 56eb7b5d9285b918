"""ctypes binding of libhplmm (argument marshalling only).

Every computation happens in the native library: Q1 assembly, partitioning
and mortar placement on the host (C++), set-up, preconditioner application
and FGMRES on the GPU (HIP).  PyTorch only provides device memory and the
stream.  The binding raises if the library is missing: there is no fallback.

torch is imported before the library is loaded so that the library binds to
the HIP runtime torch already loaded (both carry the soname libamdhip64.so.7).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libhplmm.so")

i32, i64, f64, u8 = C.c_int32, C.c_int64, C.c_double, C.c_uint8
P = C.POINTER


class HplmmSystem(C.Structure):
    _fields_ = [("n_nodes", i64), ("nnzb", i64), ("row_ptr", P(i64)), ("col_idx", P(i32)),
                ("val", P(f64)), ("rhs", P(f64)), ("node_xyz", P(i32)), ("dof_fixed", P(u8))]


class HplmmPartition(C.Structure):
    _fields_ = [("n_nodes", i64), ("n_grains", i32), ("node_grain", P(i32)), ("n_ifaces", i32), ("iface_ptr", P(i64)),
                ("iface_nodes", P(i32)), ("n_contacts", i32), ("contact_ptr", P(i64)),
                ("contact_nodes", P(i32))]


class HplmmMortar(C.Structure):
    _fields_ = [("n", i32), ("beta", f64), ("kind", i32)]


MORTAR_KINDS = {"gaussian": 0, "algebraic": 1}


class HplmmOptions(C.Structure):
    _fields_ = [("smoother_precision", i32), ("coarse_leaf_dofs", i32), ("smoother_form", i32)]


class HplmmSgStats(C.Structure):
    _fields_ = [("grains", i32), ("accepted", i32), ("fallback", i32), ("loaded", i32),
                ("max_residual_accepted", f64), ("median_residual", f64), ("t_infer_ms", f64),
                ("t_check_ms", f64), ("t_basis_ms", f64)]


class HplmmSolveInfo(C.Structure):
    _fields_ = [("iters", i32), ("rel_res_true", f64), ("t_solve_ms", f64), ("res_hist", P(f64)),
                ("res_hist_cap", i32), ("res_hist_len", i32), ("t_ml_ms", f64), ("t_mg_ms", f64)]


EXPORTS = {
    "hplmm_assemble_voxels": (i32, [i32, i32, i32, P(u8), P(f64), f64, P(f64), P(HplmmSystem)]),
    "hplmm_system_free": (None, [P(HplmmSystem)]),
    "hplmm_partition_from_voxels": (i32, [i32, i32, i32, P(u8), P(i32), i32, i32, P(HplmmPartition)]),
    "hplmm_partition_free": (None, [P(HplmmPartition)]),
    "hplmm_place_mortars": (i32, [P(i32), i32, i32, P(i32)]),
    "hplmm_plan": (i32, [P(HplmmSystem), P(HplmmPartition), P(HplmmMortar), P(HplmmOptions), C.c_void_p,
                         P(C.c_void_p)]),
    "hplmm_plan_check": (i32, [P(HplmmSystem), P(HplmmPartition), P(HplmmMortar), P(HplmmOptions), P(i64)]),
    "hplmm_setup": (i32, [C.c_void_p, C.c_void_p]),
    "hplmm_apply": (i32, [C.c_void_p, i32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "hplmm_apply_noalloc": (i32, [C.c_void_p, i32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "hplmm_spmv": (i32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "hplmm_solve": (i32, [C.c_void_p, C.c_void_p, C.c_void_p, f64, i32, i32, i32, P(HplmmSolveInfo),
                          C.c_void_p]),
    "hplmm_query": (i32, [C.c_void_p, i32, C.c_void_p, i64, P(i64)]),
    "hplmm_destroy": (None, [C.c_void_p]),
    "hplmm_profile": (i32, [C.c_void_p, i32]),
    "hplmm_use_graphs": (i32, [C.c_void_p, i32]),
    "hplmm_set_voxel_operator": (i32, [C.c_void_p, i32, i32, i32, P(u8), P(f64), f64, C.c_void_p]),
    "hplmm_debug_mortar_blocks": (i32, [C.c_void_p, C.c_void_p, C.c_void_p, P(f64), i64, P(i64)]),
    "hplmm_autotune": (i32, [C.c_void_p, i32, C.c_void_p]),
    "hplmm_set_tuning": (i32, [C.c_void_p, C.c_void_p, i64]),
    "hplmm_debug_tile_gemm": (i32, [i32, C.c_void_p, C.c_void_p, i32, C.c_void_p, C.c_void_p, i32, C.c_void_p]),
    "hplmm_debug_diag": (i32, [i32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "hplmm_stream_triad": (i32, [C.c_void_p, C.c_void_p, C.c_void_p, f64, i64, C.c_void_p]),
    "hplmm_debug_setup_stage": (i32, [C.c_void_p, i32, C.c_void_p]),
    "hplmm_debug_read_arena": (i32, [C.c_void_p, i32, i64, i64, C.c_void_p]),
    "hplmm_debug_grain_layout": (i32, [C.c_void_p, P(i64), i64]),
    "hplmm_debug_contact_layout": (i32, [C.c_void_p, P(i64), i64]),
    "hplmm_last_error": (C.c_char_p, []),
    "hplmm_sg_create": (i32, [P(i32), i32, P(C.c_void_p)]),
    "hplmm_sg_param_count": (i32, [C.c_void_p, P(i64)]),
    "hplmm_sg_set_params": (i32, [C.c_void_p, P(C.c_float), i64]),
    "hplmm_sg_get_params": (i32, [C.c_void_p, P(C.c_float), i64]),
    "hplmm_sg_forward": (i32, [C.c_void_p, C.c_void_p, i32, C.c_void_p, C.c_void_p]),
    "hplmm_sg_set_inference_precision": (i32, [C.c_void_p, i32]),
    "hplmm_sg_gradient": (i32, [C.c_void_p, C.c_void_p, C.c_void_p, i32, P(f64), C.c_void_p]),
    "hplmm_sg_get_grads": (i32, [C.c_void_p, P(C.c_float), i64, C.c_void_p]),
    "hplmm_sg_adam": (i32, [C.c_void_p, C.c_float, C.c_void_p]),
    "hplmm_sg_destroy": (None, [C.c_void_p]),
    "hplmm_sg_samples": (i32, [C.c_void_p, i64, i64, C.c_void_p, C.c_void_p, P(i32), P(i64), C.c_void_p]),
    "hplmm_setup_surrogate": (i32, [C.c_void_p, C.c_void_p, f64, C.c_void_p, C.c_void_p]),
    "hplmm_voxel_fields": (i32, [i32, i32, i32, C.c_void_p, C.c_void_p, f64, C.c_void_p, i64, C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_void_p]),
}

STATUS = {0: "OK", 1: "NOT_CONVERGED", -1: "E_ARG", -2: "E_PARTITION", -3: "E_NOT_SPD",
          -4: "E_SINGULAR_COARSE", -5: "E_HIP", -6: "E_OOM", -7: "E_NONFINITE", -8: "E_STATE"}

_lib = None


class HplmmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"hplmm {STATUS.get(code, code)}: {msg}")
        self.code = code


def lib():
    """Load libhplmm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_2509_19777_amd.build")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(code):
    if code < 0:
        raise HplmmError(code, lib().hplmm_last_error().decode())
    return code


def _ptr(a, ct):
    return a.ctypes.data_as(P(ct))


# ---- host-side problem construction ---------------------------------------------
class System:
    """Assembled fine system (numpy copies of the library's arrays)."""

    def __init__(self, n_nodes, row_ptr, col_idx, val, rhs, node_xyz, dof_fixed=None):
        self.n_nodes = int(n_nodes)
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        self.col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
        self.val = np.ascontiguousarray(val, dtype=np.float64).reshape(-1)
        self.rhs = np.ascontiguousarray(rhs, dtype=np.float64)
        self.node_xyz = np.ascontiguousarray(node_xyz, dtype=np.int32).reshape(-1)
        self.dof_fixed = None if dof_fixed is None else np.ascontiguousarray(dof_fixed, dtype=np.uint8).reshape(-1)

    @property
    def nnzb(self):
        return int(self.row_ptr[-1])

    def with_fixed(self, dof_fixed):
        """The same system with constrained dofs (uint8 / bool per dof)."""
        return System(self.n_nodes, self.row_ptr, self.col_idx, self.val, self.rhs, self.node_xyz, dof_fixed)

    def c_struct(self):
        return HplmmSystem(self.n_nodes, self.nnzb, _ptr(self.row_ptr, i64), _ptr(self.col_idx, i32),
                           _ptr(self.val, f64), _ptr(self.rhs, f64), _ptr(self.node_xyz, i32),
                           None if self.dof_fixed is None else _ptr(self.dof_fixed, u8))

    def to_scipy(self):
        """Scalar CSR matrix (for tests)."""
        import scipy.sparse as sp
        n = self.n_nodes
        blocks = self.val.reshape(-1, 3, 3)
        return sp.bsr_matrix((blocks, self.col_idx, self.row_ptr), shape=(3 * n, 3 * n)).tocsr()


def assemble_voxels(problem):
    """Q1 assembly of a synth.Problem by the library (host only)."""
    nz, ny, nx = problem.solid.shape
    solid = np.ascontiguousarray(problem.solid, dtype=np.uint8)
    E = np.ascontiguousarray(problem.E, dtype=np.float64)
    t = np.ascontiguousarray(problem.traction, dtype=np.float64)
    out = HplmmSystem()
    _check(lib().hplmm_assemble_voxels(nx, ny, nz, _ptr(solid, u8), _ptr(E, f64), float(problem.nu),
                                       _ptr(t, f64), C.byref(out)))
    try:
        n, nb = out.n_nodes, out.nnzb
        sysm = System(n, np.ctypeslib.as_array(out.row_ptr, (n + 1,)).copy(),
                      np.ctypeslib.as_array(out.col_idx, (nb,)).copy(),
                      np.ctypeslib.as_array(out.val, (9 * nb,)).copy(),
                      np.ctypeslib.as_array(out.rhs, (3 * n,)).copy(),
                      np.ctypeslib.as_array(out.node_xyz, (3 * n,)).copy())
    finally:
        lib().hplmm_system_free(C.byref(out))
    return sysm


class Partition:
    """Grains, interfaces and contact grids (numpy arrays)."""

    def __init__(self, n_grains, node_grain, iface_ptr, iface_nodes, contact_ptr, contact_nodes):
        self.n_grains = int(n_grains)
        self.node_grain = np.ascontiguousarray(node_grain, dtype=np.int32)
        self.iface_ptr = np.ascontiguousarray(iface_ptr, dtype=np.int64)
        self.iface_nodes = np.ascontiguousarray(iface_nodes, dtype=np.int32)
        self.contact_ptr = np.ascontiguousarray(contact_ptr, dtype=np.int64)
        self.contact_nodes = np.ascontiguousarray(contact_nodes, dtype=np.int32)

    @property
    def n_ifaces(self):
        return self.iface_ptr.size - 1

    @property
    def n_contacts(self):
        return self.contact_ptr.size - 1

    def iface(self, c):
        return self.iface_nodes[self.iface_ptr[c]:self.iface_ptr[c + 1]]

    def contact(self, c):
        return self.contact_nodes[self.contact_ptr[c]:self.contact_ptr[c + 1]]

    def c_struct(self):
        return HplmmPartition(self.node_grain.size, self.n_grains, _ptr(self.node_grain, i32), self.n_ifaces, _ptr(self.iface_ptr, i64),
                              _ptr(self.iface_nodes, i32), self.n_contacts, _ptr(self.contact_ptr, i64),
                              _ptr(self.contact_nodes, i32))


def partition_from_voxels(problem, w_zeta=None):
    nz, ny, nx = problem.solid.shape
    solid = np.ascontiguousarray(problem.solid, dtype=np.uint8)
    lab = np.ascontiguousarray(np.where(problem.solid > 0, problem.labels, 0), dtype=np.int32)
    w = problem.w_zeta if w_zeta is None else w_zeta
    out = HplmmPartition()
    _check(lib().hplmm_partition_from_voxels(nx, ny, nz, _ptr(solid, u8), _ptr(lab, i32), int(problem.n_grains),
                                             int(w), C.byref(out)))
    try:
        n = out.n_nodes
        nI, nC = out.n_ifaces, out.n_contacts
        ip = np.ctypeslib.as_array(out.iface_ptr, (nI + 1,)).copy()
        cp = np.ctypeslib.as_array(out.contact_ptr, (nC + 1,)).copy()
        part = Partition(out.n_grains, np.ctypeslib.as_array(out.node_grain, (n,)).copy(), ip,
                         np.ctypeslib.as_array(out.iface_nodes, (max(int(ip[-1]), 1),)).copy()[:ip[-1]],
                         cp, np.ctypeslib.as_array(out.contact_nodes, (max(int(cp[-1]), 1),)).copy()[:cp[-1]])
    finally:
        lib().hplmm_partition_free(C.byref(out))
    return part


def place_mortars(xyz, n):
    xyz = np.ascontiguousarray(xyz, dtype=np.int32).reshape(-1)
    N = xyz.size // 3
    out = np.zeros(min(n, N), dtype=np.int32)
    _check(lib().hplmm_place_mortars(_ptr(xyz, i32), N, int(n), _ptr(out, i32)))
    return out.tolist()


SMOOTHER_FORMS = {"auto": 0, "factors": 1, "inverse": 2}


def plan_check(system, part, n_mortar=2, beta=4.0, smoother_precision=64, mortar_kind="gaussian",
               coarse_leaf_dofs=0, smoother_form="auto"):
    """Host-only symbolic phase plus bounds check of every launch list."""
    s, p = system.c_struct(), part.c_struct()
    m = HplmmMortar(int(n_mortar), float(beta), MORTAR_KINDS[mortar_kind])
    o = HplmmOptions(int(smoother_precision), int(coarse_leaf_dofs), SMOOTHER_FORMS[smoother_form])
    out = np.zeros(16, dtype=np.int64)
    _check(lib().hplmm_plan_check(C.byref(s), C.byref(p), C.byref(m), C.byref(o), _ptr(out, i64)))
    keys = ["n_nodes", "nnzb", "n_grains", "n_ifaces", "n_contacts", "n_mortar", "n_corr", "n_coarse",
            "grain_mats", "ar64", "ar32", "arbf", "tile_tasks", "coarse_fronts", "coarse_levels", "max_front_dofs"]
    return dict(zip(keys, (int(x) for x in out)))


def mortar_blocks(system, part, n_mortar=2, beta=4.0, mortar_kind="gaussian"):
    """Host only: the per-interface mortar blocks of the plan, one array per
    interface (Gaussian: N_c x nu_c; algebraic: 3 N_c x 3 nu_c)."""
    s, p = system.c_struct(), part.c_struct()
    m = HplmmMortar(int(n_mortar), float(beta), MORTAR_KINDS[mortar_kind])
    need = i64(0)
    _check(lib().hplmm_debug_mortar_blocks(C.byref(s), C.byref(p), C.byref(m), None, 0, C.byref(need)))
    buf = np.zeros(max(int(need.value), 1))
    _check(lib().hplmm_debug_mortar_blocks(C.byref(s), C.byref(p), C.byref(m), _ptr(buf, f64), buf.size,
                                           C.byref(need)))
    out, off = [], 0
    for c in range(part.n_ifaces):
        Nc = int(part.iface_ptr[c + 1] - part.iface_ptr[c])
        nu = min(int(n_mortar), Nc)
        r, k = (Nc, nu) if mortar_kind == "gaussian" else (3 * Nc, 3 * nu)
        out.append(buf[off:off + r * k].reshape(r, k))
        off += r * k
    assert off == int(need.value)
    return out


# ---- device solver --------------------------------------------------------------------
def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t):
    assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
    return C.c_void_p(t.data_ptr())


class Solver:
    """hPLMM-preconditioned FGMRES on the current GPU.

    plan(...) runs the symbolic phase and uploads the inputs; setup() runs the
    numeric set-up on the device; apply/spmv/solve operate on float64 CUDA
    tensors of length 3*n_nodes.
    """

    def __init__(self, system: System, part: Partition, n_mortar=2, beta=4.0, smoother_precision=64,
                 mortar_kind="gaussian", coarse_leaf_dofs=0, smoother_form="auto"):
        if not torch.cuda.is_available():
            raise RuntimeError("hplmm.Solver needs a GPU")
        self.system, self.part = system, part
        self._keep = (system.c_struct(), part.c_struct())
        h = C.c_void_p()
        m = HplmmMortar(int(n_mortar), float(beta), MORTAR_KINDS[mortar_kind])
        o = HplmmOptions(int(smoother_precision), int(coarse_leaf_dofs), SMOOTHER_FORMS[smoother_form])
        _check(lib().hplmm_plan(C.byref(self._keep[0]), C.byref(self._keep[1]), C.byref(m), C.byref(o), _stream(),
                                C.byref(h)))
        self.h = h
        self.N = 3 * system.n_nodes
        rhs = system.rhs if system.dof_fixed is None else np.where(system.dof_fixed != 0, 0.0, system.rhs)
        self.b = torch.from_numpy(np.ascontiguousarray(rhs)).cuda()   # the load the plan uses

    def __del__(self):
        h = getattr(self, "h", None)
        if h is None or not h.value or lib is None:   # lib is None once the interpreter tears the module down
            return
        lib().hplmm_destroy(h)
        self.h = None

    def setup(self):
        _check(lib().hplmm_setup(self.h, _stream()))

    def smoother_form(self):
        """'factors' (y = W^T W x in two passes) or 'inverse' (y = S x, S = W^T W)."""
        return {1: "factors", 2: "inverse"}[int(self.query(11, np.int32)[0])]

    def set_voxel_operator(self, problem=None):
        """Matrix-free products with A from the problem's voxel grid (checked
        against the assembled matrix); None returns to the assembled operator."""
        if problem is None:
            _check(lib().hplmm_set_voxel_operator(self.h, 0, 0, 0, None, None, 0.3, _stream()))
            return
        nz, ny, nx = problem.solid.shape
        solid = np.ascontiguousarray(problem.solid, dtype=np.uint8).ravel()
        E = np.ascontiguousarray(problem.E, dtype=np.float64).ravel()
        _check(lib().hplmm_set_voxel_operator(self.h, nx, ny, nz, _ptr(solid, u8), _ptr(E, f64), float(problem.nu),
                                              _stream()))

    def use_graphs(self, on=True):
        """Replay the Arnoldi steps of the solver as HIP graphs (default on)."""
        _check(lib().hplmm_use_graphs(self.h, 1 if on else 0))

    TUNE_KEYS = ["kind", "index", "variant", "target", "waves", "t_default_us", "t_best_us"]

    def autotune(self, reps=5):
        """Time the solve-phase GEMV launch shapes on this problem and keep the
        fastest; returns the tuning records (dicts)."""
        _check(lib().hplmm_autotune(self.h, int(reps), _stream()))
        return self.tuning()

    def tuning(self):
        v = self.query(10, np.float64).reshape(-1, 7)
        return [{k: (float(x) if k.startswith("t_") else int(x)) for k, x in zip(self.TUNE_KEYS, row)} for row in v]

    def set_tuning(self, records):
        """Pin launch shapes: records as returned by autotune() / tuning()
        (kind, index, variant, waves are used); [] restores the defaults."""
        a = np.array([[r["kind"], r["index"], r["variant"], r["waves"]] for r in records], dtype=np.int32).reshape(-1, 4)
        a = np.ascontiguousarray(a)
        _check(lib().hplmm_set_tuning(self.h, a.ctypes.data_as(C.c_void_p) if a.size else None, a.shape[0]))

    def setup_surrogate(self, net, threshold):
        """Set-up with the network's shape vectors where they pass the local
        residual check (see include/hplmm_surrogate.h); returns the stats."""
        st = HplmmSgStats()
        _check(lib().hplmm_setup_surrogate(self.h, net.h, float(threshold), C.byref(st), _stream()))
        return {k: getattr(st, k) for k, _ in HplmmSgStats._fields_}

    def apply(self, r, which=0, out=None):
        z = torch.empty_like(r) if out is None else out
        _check(lib().hplmm_apply(self.h, int(which), _dptr(r), _dptr(z), _stream()))
        return z

    def apply_noalloc(self, r, which=0, out=None):
        """hplmm_apply_noalloc: the same application with the library's static
        split-row scratch; allocates nothing in the library (out must be given
        for an allocation-free call from Python)."""
        z = torch.empty_like(r) if out is None else out
        _check(lib().hplmm_apply_noalloc(self.h, int(which), _dptr(r), _dptr(z), _stream()))
        return z

    def split_scratch(self):
        """Partial sums (doubles) the coarse sweeps' split rows need."""
        v = self.query(12, np.int64)
        return int(v[0])

    def spmv(self, x, out=None):
        y = torch.empty_like(x) if out is None else out
        _check(lib().hplmm_spmv(self.h, _dptr(x), _dptr(y), _stream()))
        return y

    def solve(self, b=None, x0=None, rtol=1e-8, restart=50, maxit=300, fixed_iters=0, hist_cap=1024):
        b = self.b if b is None else b
        x = torch.zeros_like(b) if x0 is None else x0.clone()
        hist = np.zeros(hist_cap)
        info = HplmmSolveInfo(0, 0.0, 0.0, _ptr(hist, f64), hist_cap, 0, 0.0, 0.0)
        code = _check(lib().hplmm_solve(self.h, _dptr(b), _dptr(x), float(rtol), int(restart), int(maxit),
                                        int(fixed_iters), C.byref(info), _stream()))
        return x, {"status": STATUS[code], "iters": info.iters, "rel_res": info.rel_res_true,
                   "t_solve_ms": info.t_solve_ms, "t_ml_ms": info.t_ml_ms, "t_mg_ms": info.t_mg_ms,
                   "history": hist[:info.res_hist_len].copy()}

    def query(self, what, dtype):
        need = i64(0)
        _check(lib().hplmm_query(self.h, int(what), None, 0, C.byref(need)))
        buf = np.zeros(max(int(need.value), 1), dtype=np.uint8)
        _check(lib().hplmm_query(self.h, int(what), buf.ctypes.data_as(C.c_void_p), buf.size, C.byref(need)))
        return buf[:need.value].view(dtype)

    def sizes(self):
        keys = ["n_nodes", "nnzb", "n_grains", "n_ifaces", "n_contacts", "n_mortar", "n_corr", "n_coarse",
                "grain_mats", "max_grain_dofs", "max_contact_dofs", "sell_slices", "sell_padded_blocks",
                "coarse_fronts", "coarse_levels", "max_front_dofs"]
        v = self.query(0, np.int64)
        return dict(zip(keys, (int(x) for x in v)))

    def coarse_matrix(self):
        n = self.sizes()["n_coarse"]
        return self.query(4, np.float64).reshape(n, n)

    PROF_CLASSES = ["tile_gemm", "diag", "gemv_smoother", "gemv_coarse", "gemv_basis", "spmv", "apply",
                    "smoother_reduce"]

    def profile(self, classes):
        """Enable event timing for the named kernel classes (empty: off)."""
        mask = 0
        for c in classes:
            mask |= 1 << self.PROF_CLASSES.index(c)
        _check(lib().hplmm_profile(self.h, mask))

    def profile_results(self):
        v = self.query(7, np.float64).reshape(-1, 3)
        return {name: {"launches": int(v[i, 0]), "ms": float(v[i, 1]), "units": float(v[i, 2])}
                for i, name in enumerate(self.PROF_CLASSES)}

    def algorithmic_bytes(self):
        v = self.query(8, np.float64)
        return {"apply": float(v[0]), "spmv": float(v[1])}

    def method_work(self):
        """The method's own work (query 13): set-up flops from unpadded sizes,
        the flops the set-up's tile tasks issue, and the bytes one M^-1
        application needs with every operator read once."""
        v = self.query(13, np.float64)
        k4 = ["grains", "contacts", "coarse", "total"]
        return {"setup_flops": dict(zip(k4, map(float, v[0:4]))),
                "issued_setup_flops": dict(zip(k4, map(float, v[4:8]))),
                "apply_bytes": dict(zip(["smoother", "basis", "coarse", "spmv", "total"], map(float, v[8:13])))}

    def setup_times_ms(self):
        v = self.query(5, np.float64)
        return {"grains": v[0], "contacts": v[1], "coarse": v[2], "total": v[3]}


# ---- test hooks ---------------------------------------------------------------
def _vp(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def debug_tile_gemm(A, B, C_, flags, P_=None, npairs=None):
    """One tile task on CUDA tensors: A, B (npairs, 64, 64) as column-major tiles
    (i.e. tensors holding the transposed tile), C_ (64, 64) updated in place.
    npairs defaults to A.shape[0]; 0 is allowed with the right-factor flag."""
    prec = {torch.float64: 64, torch.float32: 32, torch.int16: 16}[A.dtype]   # int16: bfloat16 bits
    n = int(A.shape[0]) if npairs is None else int(npairs)
    if n > A.shape[0] or n > B.shape[0]:
        raise ValueError("npairs exceeds the tiles given")
    _check(lib().hplmm_debug_tile_gemm(prec, _vp(A), _vp(B), n, _vp(P_), _vp(C_), int(flags), _stream()))


def debug_diag(A, P=None):
    prec = 64 if A.dtype == torch.float64 else 32
    if P is not None and (P.dtype != A.dtype or P.numel() != A.numel() or not P.is_contiguous()):
        raise ValueError("P must be one contiguous tile of A's type")
    W = torch.empty_like(A)
    Wt = torch.empty_like(A)
    _check(lib().hplmm_debug_diag(prec, _vp(A), _vp(P), _vp(W), _vp(Wt), _stream()))
    return A, W, Wt


def stream_triad(a, b, c, scalar):
    """a = b + scalar c on float64 device tensors (the bandwidth reference)."""
    for t in (a, b, c):
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise ValueError("triad arrays must be contiguous float64 device tensors")
    if not (a.numel() == b.numel() == c.numel()):
        raise ValueError("triad arrays must have one length")
    _check(lib().hplmm_stream_triad(_vp(a), _vp(b), _vp(c), float(scalar), a.numel(), _stream()))
    return a


def debug_setup_stage(solver, stage):
    _check(lib().hplmm_debug_setup_stage(solver.h, int(stage), _stream()))


def debug_read_arena(solver, arena, off, count):
    dt = {0: np.float64, 1: np.float32, 2: np.uint16}[arena]
    out = np.zeros(int(count), dtype=dt)
    _check(lib().hplmm_debug_read_arena(solver.h, int(arena), int(off), int(count), out.ctypes.data_as(C.c_void_p)))
    return out


def debug_grain_layout(solver):
    nm = solver.sizes()["grain_mats"]
    out = np.zeros(11 * nm, dtype=np.int64)
    _check(lib().hplmm_debug_grain_layout(solver.h, _ptr(out, i64), out.size))
    return out.reshape(nm, 11)


def debug_contact_layout(solver):
    nm = solver.sizes()["n_contacts"]
    out = np.zeros(6 * nm, dtype=np.int64)
    _check(lib().hplmm_debug_contact_layout(solver.h, _ptr(out, i64), out.size))
    return out.reshape(nm, 6)


def debug_read_lower(solver, arena, off, n, nt):
    """The packed lower tiles of an n x n block at arena offset off (tiles
    column-major inside, (I, J) at I (I + 1) / 2 + J) as a dense lower
    triangular float64 array."""
    v = debug_read_arena(solver, arena, off, nt * (nt + 1) // 2 * 4096).astype(np.float64)
    M = np.zeros((nt * 64, nt * 64))
    for I in range(nt):
        for J in range(I + 1):
            t = v[(I * (I + 1) // 2 + J) * 4096:(I * (I + 1) // 2 + J + 1) * 4096].reshape(64, 64).T
            M[I * 64:(I + 1) * 64, J * 64:(J + 1) * 64] = t
    return np.tril(M[:n, :n])


class VoxelGrid:
    """A problem's voxel grid on the device with the library's node numbering
    (lattice point -> free node from System.node_xyz), for hplmm_voxel_fields."""

    def __init__(self, problem, system):
        nz, ny, nx = problem.solid.shape
        self.dims = (nx, ny, nz)
        self.nu = float(problem.nu)
        self.n_nodes = system.n_nodes
        xyz = system.node_xyz.reshape(-1, 3).astype(np.int64)
        lat = -np.ones((nx + 1) * (ny + 1) * (nz + 1), dtype=np.int32)
        lat[xyz[:, 0] + (nx + 1) * (xyz[:, 1] + (ny + 1) * xyz[:, 2])] = np.arange(system.n_nodes, dtype=np.int32)
        self.solid = torch.from_numpy(np.ascontiguousarray(problem.solid, dtype=np.uint8).ravel()).cuda()
        self.E = torch.from_numpy(np.ascontiguousarray(problem.E, dtype=np.float64).ravel()).cuda()
        self.lat2node = torch.from_numpy(lat).cuda()
        self.mask = self.solid.bool()

    def fields(self, x):
        """(sigma_t [n_vox], u_centroid [n_vox, 3]) of the displacement x (device)."""
        nx, ny, nz = self.dims
        nv = nx * ny * nz
        st = torch.empty(nv, dtype=torch.float64, device=x.device)
        uc = torch.empty(3 * nv, dtype=torch.float64, device=x.device)
        _check(lib().hplmm_voxel_fields(nx, ny, nz, _vp(self.solid), _vp(self.E), self.nu, _vp(self.lat2node),
                                        self.n_nodes, _vp(x), _vp(st), _vp(uc), _stream()))
        return st, uc.view(nv, 3)


def build_problem(problem, w_zeta=None):
    """Assemble and partition a synth.Problem with the library (host only)."""
    return assemble_voxels(problem), partition_from_voxels(problem, w_zeta)


# ---- learned basis surrogate network ------------------------------------------------
class SurrogateNet:
    """The 3D convolutional basis surrogate (see include/hplmm_surrogate.h).

    Parameters are exchanged as one float32 vector in the library's order:
    per layer w[d][ci][co] then b[co].  Inputs and targets are CUDA float32
    tensors shaped (n, 9, 9, 9, c) (channel-last)."""

    def __init__(self, channels=(4, 32, 32, 32, 9), max_batch=256):
        self.channels = tuple(int(c) for c in channels)
        self.max_batch = int(max_batch)
        ch = (i32 * 5)(*self.channels)
        h = C.c_void_p()
        _check(lib().hplmm_sg_create(ch, self.max_batch, C.byref(h)))
        self.h = h
        n = i64(0)
        _check(lib().hplmm_sg_param_count(self.h, C.byref(n)))
        self.n_params = int(n.value)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is None or not h.value or lib is None:   # lib is None once the interpreter tears the module down
            return
        lib().hplmm_sg_destroy(h)
        self.h = None

    def set_params(self, flat):
        a = np.ascontiguousarray(flat, dtype=np.float32)
        _check(lib().hplmm_sg_set_params(self.h, a.ctypes.data_as(P(C.c_float)), a.size))

    def get_params(self):
        a = np.zeros(self.n_params, dtype=np.float32)
        _check(lib().hplmm_sg_get_params(self.h, a.ctypes.data_as(P(C.c_float)), a.size))
        return a

    def forward(self, x, out=None):
        n = x.shape[0]
        y = torch.empty((n, 9, 9, 9, self.channels[-1]), dtype=torch.float32, device=x.device) if out is None else out
        _check(lib().hplmm_sg_forward(self.h, _vp(x), int(n), _vp(y), _stream()))
        return y

    def set_inference_precision(self, precision):
        """32 (float32) or 16 (bfloat16 operands, float32 accumulation) for
        forward() and the set-up's predictions; training stays float32."""
        _check(lib().hplmm_sg_set_inference_precision(self.h, int(precision)))

    def gradient(self, x, y):
        loss = f64(0.0)
        _check(lib().hplmm_sg_gradient(self.h, _vp(x), _vp(y), int(x.shape[0]), C.byref(loss), _stream()))
        return float(loss.value)

    def get_grads(self):
        a = np.zeros(self.n_params, dtype=np.float32)
        _check(lib().hplmm_sg_get_grads(self.h, a.ctypes.data_as(P(C.c_float)), a.size, _stream()))
        return a

    def adam(self, lr):
        _check(lib().hplmm_sg_adam(self.h, C.c_float(lr), _stream()))


def flatten_params(params):
    """[(w (3,3,3,ci,co), b (co,)), ...] -> one float32 vector in the library's order."""
    return np.concatenate([np.concatenate([w.reshape(-1), b.reshape(-1)]) for w, b in params]).astype(np.float32)


def unflatten_params(flat, channels):
    out, o = [], 0
    for ci, co in zip(channels[:-1], channels[1:]):
        nw = 27 * ci * co
        out.append((np.asarray(flat[o:o + nw], dtype=np.float64).reshape(3, 3, 3, ci, co),
                    np.asarray(flat[o + nw:o + nw + co], dtype=np.float64)))
        o += nw + co
    return out


def surrogate_samples(solver, first=0, count=None, targets=True):
    """Network inputs (and exact targets) of a Solver's (grain, interface,
    mortar) samples as CUDA float32 tensors (n, 9, 9, 9, 4) / (n, 9, 9, 9, 9),
    plus the (n, 3) int32 meta array {grain matrix, interface, mortar}."""
    total = i64(0)
    _check(lib().hplmm_sg_samples(solver.h, 0, 0, None, None, None, C.byref(total), _stream()))
    n = int(total.value) - first if count is None else int(count)
    x = torch.empty((n, 9, 9, 9, 4), dtype=torch.float32, device="cuda")
    y = torch.empty((n, 9, 9, 9, 9), dtype=torch.float32, device="cuda") if targets else None
    meta = np.zeros((n, 3), dtype=np.int32)
    _check(lib().hplmm_sg_samples(solver.h, int(first), n, _vp(x), _vp(y), meta.ctypes.data_as(P(i32)), None,
                                  _stream()))
    return x, y, meta
