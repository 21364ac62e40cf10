"""Python binding of the HIP library (``_lib/libhps.so``, C ABI in ``include/hps.h``).

Argument marshalling only: every step of the solver runs in the library's HIP
kernels.  PyTorch supplies device memory (one ``uint8`` workspace tensor per
problem, plus the input/output tensors) and the stream.  Importing this module
fails loudly when the library has not been built; there is no fallback.

Vectors use the canonical skeleton layout of ``include/hps.h``: complex128
tensors of length n*n*4*(N-1), slot (e, side, k) at (e*4 + side)*(N-1) + k.
"""
import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libhps.so")

HPS_OK, HPS_NOT_CONVERGED = 0, 1
HPS_ERR = {-1: "HPS_ERR_ARG", -2: "HPS_ERR_OOM", -3: "HPS_ERR_SINGULAR",
           -4: "HPS_ERR_STATE", -5: "HPS_ERR_HIP"}
HPS_FP64, HPS_MIXED = 0, 1
HPS_OPT_GRAPHS, HPS_OPT_TIMING = 1, 2
HPS_KERNEL_LEAF = 0


class HPSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{HPS_ERR.get(code, code)}: {msg}")
        self.code = code


class Desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("order", ctypes.c_int32),
                ("kappa", ctypes.c_double), ("eta", ctypes.c_double),
                ("precision", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("coarse_iters", ctypes.c_int32), ("gamma", ctypes.c_int32),
                ("restart", ctypes.c_int32), ("ny", ctypes.c_int32)]


def mesh_dims(desc):
    """(nx, ny) elements of a descriptor (ny 0: the square n x n mesh)."""
    return desc.n, (desc.ny or desc.n)


class Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("relres_est", ctypes.c_double), ("relres_true", ctypes.c_double),
                ("t_build_s", ctypes.c_double), ("t_solve_s", ctypes.c_double)]


class LevelView(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("boxes", ctypes.c_int32),
                ("box_nodes", ctypes.c_int32), ("morton", ctypes.c_int32),
                ("T", ctypes.c_void_p), ("pairs", ctypes.c_int32),
                ("shared_nodes", ctypes.c_int32), ("Ainv", ctypes.c_void_p),
                ("X", ctypes.c_void_p), ("fp32", ctypes.c_int32)]


_P = ctypes.c_void_p
_PP = ctypes.POINTER(ctypes.c_void_p)
_SIGS = {
    "hps_ctx_create": ([_P, ctypes.POINTER(_P)], ctypes.c_int),
    "hps_ctx_destroy": ([_P], ctypes.c_int),
    "hps_last_error": ([_P], ctypes.c_char_p),
    "hps_sync": ([_P], ctypes.c_int),
    "hps_set_option": ([_P, ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
    "hps_kernel_time": ([_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                         ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "hps_workspace_bytes": ([ctypes.POINTER(Desc), ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "hps_gll_nodes": ([ctypes.c_int32, _P], ctypes.c_int),
    "hps_node_coords": ([ctypes.POINTER(Desc), _P, _P], ctypes.c_int),
    "hps_slot_coords": ([ctypes.POINTER(Desc), _P, _P, _P, _P], ctypes.c_int),
    "hps_problem_create": ([_P, ctypes.POINTER(Desc), _P, ctypes.c_size_t, ctypes.POINTER(_P)],
                           ctypes.c_int),
    "hps_problem_destroy": ([_P], ctypes.c_int),
    "hps_level_view_get": ([_P, ctypes.c_int32, ctypes.POINTER(LevelView)], ctypes.c_int),
    "hps_member_level_view": ([_P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(LevelView)], ctypes.c_int),
    "hps_group_workspace_bytes": ([ctypes.POINTER(Desc), ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)],
                                  ctypes.c_int),
    "hps_group_create": ([_P, ctypes.POINTER(Desc), ctypes.c_int32, _P, _P, _P, ctypes.c_size_t,
                          ctypes.POINTER(_P)], ctypes.c_int),
    "hps_group_size": ([_P], ctypes.c_int32),
    "hps_leaf_maps_noalloc": ([_P, ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                               ctypes.c_int32, _P, _P, _P, _P], ctypes.c_int),
    "hps_choose_levels": ([ctypes.POINTER(Desc), ctypes.c_int32, ctypes.c_size_t, ctypes.POINTER(ctypes.c_int32)],
                          ctypes.c_int),
    "hps_build_leaves": ([_PP, ctypes.c_int32, _PP, _PP], ctypes.c_int),
    "hps_merge_level": ([_PP, ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
    "hps_set_rhs": ([_PP, ctypes.c_int32, _PP, _PP], ctypes.c_int),
    "hps_skeleton_apply": ([_PP, ctypes.c_int32, ctypes.c_int32, _PP, _PP], ctypes.c_int),
    "hps_precond_apply": ([_PP, ctypes.c_int32, _PP, _PP], ctypes.c_int),
    "hps_recover_field": ([_PP, ctypes.c_int32, _PP, _PP, _PP, _PP, _PP], ctypes.c_int),
    "hps_gmres_solve": ([_PP, ctypes.c_int32, _PP, _PP, ctypes.c_double, ctypes.c_int32,
                         ctypes.POINTER(Info)], ctypes.c_int),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} is missing "
                          "(run `python -m paper_2511_00735_amd.build`)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (args, res) in _SIGS.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


lib = _load()


def _ptrs(values):
    arr = (ctypes.c_void_p * len(values))(*values)
    return ctypes.cast(arr, _PP)


def _dptr(t):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous CUDA tensor")
    return t.data_ptr()


def make_desc(n, order, kappa, eta=None, levels=0, coarse_iters=5, restart=60,
              precision=HPS_FP64, gamma=1, ny=0):
    """n: elements along x (n x n when ny is 0); ny: elements along y."""
    return Desc(n, order, float(kappa), float(kappa if eta is None else eta), precision,
                levels, coarse_iters, gamma, restart, ny)


def workspace_bytes(desc):
    out = ctypes.c_size_t(0)
    rc = lib.hps_workspace_bytes(ctypes.byref(desc), ctypes.byref(out))
    if rc != HPS_OK:
        raise HPSError(rc, "invalid descriptor")
    return out.value


def leaf_maps_noalloc(ctx, order, h, kappa, eta, b_nodes, s_nodes, T, H):
    """Leaf maps of b_nodes.shape[0] elements into T ([E][4p][4p] column-major)
    and H ([E][4p]) with no device allocation (the library's static scratch)."""
    count = b_nodes.shape[0]
    ctx.check(lib.hps_leaf_maps_noalloc(ctx.handle, order, float(h), float(kappa), float(eta), count,
                                        _dptr(b_nodes), _dptr(s_nodes), _dptr(T), _dptr(H)),
              "hps_leaf_maps_noalloc")


def choose_levels(desc, budget, count=1):
    """Most levels L whose workspace for `count` problems fits `budget` bytes."""
    out = ctypes.c_int32(0)
    rc = lib.hps_choose_levels(ctypes.byref(desc), count, ctypes.c_size_t(int(budget)), ctypes.byref(out))
    if rc != HPS_OK:
        raise HPSError(rc, f"no level count fits {budget} bytes")
    return out.value


def gll_nodes(order):
    xi = np.zeros(order + 1)
    rc = lib.hps_gll_nodes(order, xi.ctypes.data)
    if rc != HPS_OK:
        raise HPSError(rc, "hps_gll_nodes")
    return xi


def node_coords(desc):
    nx, ny = mesh_dims(desc)
    E, N1 = nx * ny, desc.order + 1
    x = np.zeros(E * N1 * N1)
    y = np.zeros(E * N1 * N1)
    rc = lib.hps_node_coords(ctypes.byref(desc), x.ctypes.data, y.ctypes.data)
    if rc != HPS_OK:
        raise HPSError(rc, "hps_node_coords")
    return x.reshape(E, N1 * N1), y.reshape(E, N1 * N1)


def slot_coords(desc):
    nx, ny = mesh_dims(desc)
    ns = nx * ny * 4 * (desc.order - 1)
    arrs = [np.zeros(ns) for _ in range(4)]
    rc = lib.hps_slot_coords(ctypes.byref(desc), *[a.ctypes.data for a in arrs])
    if rc != HPS_OK:
        raise HPSError(rc, "hps_slot_coords")
    return tuple(arrs)


class Context:
    """A library context bound to a torch CUDA stream (default: current stream)."""

    def __init__(self, stream=None):
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        rc = lib.hps_ctx_create(ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc != HPS_OK:
            raise HPSError(rc, "hps_ctx_create")
        self.handle = h

    def check(self, rc, what):
        if rc < 0:
            msg = lib.hps_last_error(self.handle)
            raise HPSError(rc, f"{what}: {msg.decode() if msg else ''}")
        return rc

    def sync(self):
        self.check(lib.hps_sync(self.handle), "hps_sync")

    def set_graphs(self, on):
        """Replay captured HIP graphs (each FGMRES iteration of a solve, and the V-cycle of
        precond_apply), or launch eagerly (the default)."""
        self.check(lib.hps_set_option(self.handle, HPS_OPT_GRAPHS, 1 if on else 0), "hps_set_option")

    def set_timing(self, on):
        """Bracket launches of the timed kernels with HIP events (discards old records)."""
        self.check(lib.hps_set_option(self.handle, HPS_OPT_TIMING, 1 if on else 0), "hps_set_option")

    def kernel_time(self, kernel=None):
        """(launches, summed device ms, units) of a timed kernel since set_timing."""
        kernel = HPS_KERNEL_LEAF if kernel is None else kernel
        n, ms, u = ctypes.c_int64(), ctypes.c_double(), ctypes.c_int64()
        self.check(lib.hps_kernel_time(self.handle, kernel, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(u)),
                   "hps_kernel_time")
        return n.value, ms.value, u.value

    def __del__(self):
        if getattr(self, "handle", None) and lib is not None:
            lib.hps_ctx_destroy(self.handle)
            self.handle = None


class Problem:
    """One Helmholtz problem living in one device workspace."""

    def __init__(self, ctx, desc, workspace=None):
        self.ctx = ctx
        self.desc = desc
        self.n, self.N = desc.n, desc.order
        self.nx, self.ny = mesh_dims(desc)
        self.p = self.N - 1
        self.E = self.nx * self.ny
        self.nslots = self.E * 4 * self.p
        self.bytes = workspace_bytes(desc)
        if workspace is None:
            workspace = torch.empty(self.bytes + 256, dtype=torch.uint8, device="cuda")
        self._ws_tensor = workspace
        base = workspace.data_ptr()
        self.ws_offset = (-base) % 256
        h = ctypes.c_void_p()
        ctx.check(lib.hps_problem_create(ctx.handle, ctypes.byref(desc),
                                         ctypes.c_void_p(base + self.ws_offset),
                                         ctypes.c_size_t(workspace.numel() - self.ws_offset),
                                         ctypes.byref(h)), "hps_problem_create")
        self.handle = h
        self.count = 1
        self.lmax = int(round(np.log2(self.nx))) + int(round(np.log2(self.ny)))
        self.levels = desc.levels or self.lmax

    def __del__(self):
        if getattr(self, "handle", None) and lib is not None:
            lib.hps_problem_destroy(self.handle)
            self.handle = None

    # ---- data preparation (problem inputs, evaluated at the library's nodes)
    def coefficient_nodes(self, b_fn):
        x, y = node_coords(self.desc)
        return torch.from_numpy(np.ascontiguousarray(b_fn(x, y), dtype=np.float64)).cuda()

    def source_nodes(self, s_fn):
        x, y = node_coords(self.desc)
        return torch.from_numpy(np.ascontiguousarray(s_fn(x, y), dtype=np.complex128)).cuda()

    def boundary_data(self, t_fn):
        x, y, nx, ny = slot_coords(self.desc)
        return torch.from_numpy(np.ascontiguousarray(t_fn(x, y, nx, ny), dtype=np.complex128)).cuda()

    # ---- hot path ---------------------------------------------------------
    def build_leaves(self, b_nodes, s_nodes=None):
        build_leaves([self], [b_nodes], None if s_nodes is None else [s_nodes])

    def merge_level(self, level):
        merge_level([self], level)

    def merge_all(self):
        top = self.levels if self.desc.coarse_iters == -1 else self.levels - 1
        for level in range(1, top + 1):
            self.merge_level(level)

    def set_rhs(self, t):
        rhs = torch.empty(self.nslots, dtype=torch.complex128, device="cuda")
        set_rhs([self], [t], [rhs])
        return rhs

    def skeleton_apply(self, g, level=1, out=None):
        if out is None:
            out = torch.zeros(self.nslots, dtype=torch.complex128, device="cuda")
        p = _ptrs([self.handle.value])
        self.ctx.check(lib.hps_skeleton_apply(p, 1, level, _ptrs([_dptr(g)]), _ptrs([_dptr(out)])),
                       "hps_skeleton_apply")
        return out

    def precond_apply(self, r, out=None):
        if out is None:
            out = torch.empty(self.nslots, dtype=torch.complex128, device="cuda")
        precond_apply([self], [r], [out])
        return out

    def gmres_solve(self, rhs, tol=1e-10, maxit=600, out=None):
        if out is None:
            out = torch.empty(self.nslots, dtype=torch.complex128, device="cuda")
        infos = gmres_solve([self], [rhs], [out], tol, maxit)
        return out, infos[0]

    def recover_field(self, b_nodes, t, g, s_nodes=None):
        """Nodal field u [E, (N+1)^2] of every element from the solution g."""
        u = torch.empty((self.E, (self.N + 1) ** 2), dtype=torch.complex128, device="cuda")
        recover_field([self], [b_nodes], None if s_nodes is None else [s_nodes], [t], [g], [u])
        return u

    # ---- inspection -------------------------------------------------------
    def level_view(self, level):
        v = LevelView()
        self.ctx.check(lib.hps_level_view_get(self.handle, level, ctypes.byref(v)), "level_view")
        return v

    def _view(self, ptr, count, fp32=False):
        off = ptr - self._ws_tensor.data_ptr()
        size = 8 if fp32 else 16
        raw = self._ws_tensor[off:off + size * count]
        return raw.view(torch.complex64 if fp32 else torch.complex128)

    def level_T(self, level):
        """Box maps of a level as [boxes, b, b] (row, column), Morton box order
        (complex64 for the FP32 levels of mixed precision)."""
        v = self.level_view(level)
        b = v.box_nodes
        t = self._view(v.T, v.boxes * b * b, bool(v.fp32)).view(v.boxes, b, b)
        return t.transpose(1, 2)   # stored column-major

    def level_Ainv(self, level):
        """Per-pair A^-1 as [pairs, 2m, 2m] (x = [Q.beta; P.alpha]), or None."""
        v = self.level_view(level)
        m2 = 2 * v.shared_nodes
        if not v.Ainv:
            return None
        return self._view(v.Ainv, v.pairs * m2 * m2, bool(v.fp32)).view(v.pairs, m2, m2).transpose(1, 2)

    def level_X(self, level):
        """Per-pair X = A^-1 B as [pairs, 2m, 2e] (columns y = [P.E1; Q.E2]), or None."""
        v = self.level_view(level)
        if not v.X:
            return None
        m2 = 2 * v.shared_nodes
        e2 = 2 * (v.box_nodes - v.shared_nodes)
        return self._view(v.X, v.pairs * m2 * e2, bool(v.fp32)).view(v.pairs, e2, m2).transpose(1, 2)


def group_workspace_bytes(desc, count):
    b = ctypes.c_size_t()
    rc = lib.hps_group_workspace_bytes(ctypes.byref(desc), count, ctypes.byref(b))
    if rc != HPS_OK:
        raise HPSError(rc, "hps_group_workspace_bytes")
    return b.value


class Group:
    """`count` problems of one shape (kappa and eta per problem) batched in
    every hot-path launch; per-problem inputs and outputs are lists."""

    def __init__(self, ctx, desc, kappas, etas=None, workspace=None):
        kappas = [float(k) for k in kappas]
        etas = list(kappas) if etas is None else [float(e) for e in etas]
        self.ctx = ctx
        self.desc = desc
        self.count = len(kappas)
        self.n, self.N = desc.n, desc.order
        self.nx, self.ny = mesh_dims(desc)
        self.p = self.N - 1
        self.E = self.nx * self.ny
        self.nslots = self.E * 4 * self.p
        self.lmax = int(round(np.log2(self.nx))) + int(round(np.log2(self.ny)))
        self.levels = desc.levels or self.lmax
        self.bytes = group_workspace_bytes(desc, self.count)
        if workspace is None:
            workspace = torch.empty(self.bytes + 256, dtype=torch.uint8, device="cuda")
        self._ws_tensor = workspace
        base = workspace.data_ptr()
        off = (-base) % 256
        ka = (ctypes.c_double * self.count)(*kappas)
        ea = (ctypes.c_double * self.count)(*etas)
        h = ctypes.c_void_p()
        ctx.check(lib.hps_group_create(ctx.handle, ctypes.byref(desc), self.count, ka, ea,
                                       ctypes.c_void_p(base + off), ctypes.c_size_t(workspace.numel() - off),
                                       ctypes.byref(h)), "hps_group_create")
        self.handle = h

    def __del__(self):
        if getattr(self, "handle", None) and lib is not None:
            lib.hps_problem_destroy(self.handle)
            self.handle = None

    def build_leaves(self, b_nodes, s_nodes=None):
        build_leaves([self], b_nodes, s_nodes)

    def merge_all(self):
        top = self.levels if self.desc.coarse_iters == -1 else self.levels - 1
        for level in range(1, top + 1):
            merge_level([self], level)

    def set_rhs(self, ts):
        rhs = [torch.empty(self.nslots, dtype=torch.complex128, device="cuda") for _ in ts]
        set_rhs([self], ts, rhs)
        return rhs

    def precond_apply(self, rs):
        zs = [torch.empty(self.nslots, dtype=torch.complex128, device="cuda") for _ in rs]
        precond_apply([self], rs, zs)
        return zs

    def gmres_solve(self, rhs, tol=1e-10, maxit=600, out=None):
        out = out if out is not None else [torch.empty(self.nslots, dtype=torch.complex128, device="cuda")
                                           for _ in rhs]
        infos = gmres_solve([self], rhs, out, tol, maxit)
        return out, infos

    def member_view(self, member, level):
        v = LevelView()
        self.ctx.check(lib.hps_member_level_view(self.handle, member, level, ctypes.byref(v)), "member view")
        return v

    def level_T(self, member, level):
        v = self.member_view(member, level)
        b = v.box_nodes
        off = v.T - self._ws_tensor.data_ptr()
        size = 8 if v.fp32 else 16
        raw = self._ws_tensor[off:off + size * v.boxes * b * b]
        t = raw.view(torch.complex64 if v.fp32 else torch.complex128).view(v.boxes, b, b)
        return t.transpose(1, 2)


# ---- batch-first entry points (several problems per call) ------------------
def _handles(problems):
    return _ptrs([p.handle.value for p in problems])


def _nprob(problems, *arrays):
    """Problems behind the handles; every per-problem array must list them all."""
    total = sum(p.count for p in problems)
    for a in arrays:
        if a is not None and len(a) != total:
            raise ValueError(f"per-problem array has {len(a)} entries for {total} problems")
    return total


def build_leaves(problems, b_nodes, s_nodes=None):
    _nprob(problems, b_nodes, s_nodes)
    ctx = problems[0].ctx
    s = _ptrs([_dptr(x) for x in s_nodes]) if s_nodes is not None else None
    ctx.check(lib.hps_build_leaves(_handles(problems), len(problems),
                                   _ptrs([_dptr(b) for b in b_nodes]), s), "hps_build_leaves")


def merge_level(problems, level):
    problems[0].ctx.check(lib.hps_merge_level(_handles(problems), len(problems), level),
                          "hps_merge_level")


def set_rhs(problems, t, rhs):
    _nprob(problems, t, rhs)
    problems[0].ctx.check(lib.hps_set_rhs(_handles(problems), len(problems),
                                          _ptrs([_dptr(x) for x in t]),
                                          _ptrs([_dptr(x) for x in rhs])), "hps_set_rhs")


def precond_apply(problems, r, z):
    _nprob(problems, r, z)
    problems[0].ctx.check(lib.hps_precond_apply(_handles(problems), len(problems),
                                                _ptrs([_dptr(x) for x in r]),
                                                _ptrs([_dptr(x) for x in z])), "hps_precond_apply")


def recover_field(problems, b_nodes, s_nodes, t, g, u):
    _nprob(problems, b_nodes, s_nodes, t, g, u)
    s = _ptrs([_dptr(x) for x in s_nodes]) if s_nodes is not None else None
    problems[0].ctx.check(lib.hps_recover_field(_handles(problems), len(problems),
                                                _ptrs([_dptr(x) for x in b_nodes]), s,
                                                _ptrs([_dptr(x) for x in t]), _ptrs([_dptr(x) for x in g]),
                                                _ptrs([_dptr(x) for x in u])), "hps_recover_field")


def gmres_solve(problems, rhs, g, tol=1e-10, maxit=600):
    infos = (Info * _nprob(problems, rhs, g))()
    problems[0].ctx.check(lib.hps_gmres_solve(_handles(problems), len(problems),
                                              _ptrs([_dptr(x) for x in rhs]),
                                              _ptrs([_dptr(x) for x in g]), tol, maxit, infos),
                          "hps_gmres_solve")
    return [dict(status=i.status, iterations=i.iterations, relres_est=i.relres_est,
                 relres_true=i.relres_true, t_build_s=i.t_build_s, t_solve_s=i.t_solve_s) for i in infos]


def tree_box_xy(level, j, nx=None, ny=None):
    """(bx, by) of box j of a level in the library's merge-tree storage order on
    an nx x ny mesh (None: a square mesh, where the order is the Morton order).
    Bit l-1 of an element's tree code is the next unused bit of its x index if
    merge l runs along x, else of its y index."""
    ax = ay = 64
    if nx is not None:
        ax, ay = int(round(np.log2(nx))), int(round(np.log2(ny)))
    c = min(ax, ay)
    code = j << (level - 1)
    ex = ey = dx = dy = 0
    for bit in range(40):
        l = bit + 1
        along_x = (l % 2 == 1) if l <= 2 * c else ax > ay
        if along_x:
            ex |= ((code >> bit) & 1) << dx
            dx += 1
        else:
            ey |= ((code >> bit) & 1) << dy
            dy += 1
    # merges along x and y before this level
    mx = sum(1 for l in range(1, level) if ((l % 2 == 1) if l <= 2 * c else ax > ay))
    my = (level - 1) - mx
    return ex >> mx, ey >> my


def morton_box_xy(level, j):
    """(bx, by) of box j of a level of a square mesh (merge-tree = Morton order)."""
    return tree_box_xy(level, j)