"""hpdg: MI355X-native matrix-free SIPG hp-DG operator and multigrid-preconditioned solve.

Thin ctypes binding of the C ABI in ``include/hpdg.h`` (libhpdg.so, HIP kernels for
gfx950).  The binding only marshals arguments: every step of the operator, smoother,
V-cycle and Krylov solve runs in the library's kernels.  Device vectors are torch CUDA
(ROCm) tensors; streams are torch streams.  Importing this package fails loudly when
the library has not been built (``python -m paper_1907_01572_amd.build``).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhpdg.so")

OK = 0
ERR_INVALID_ARG, ERR_INVALID_MESH, ERR_OOM, ERR_NOT_CONVERGED, ERR_BREAKDOWN, ERR_HIP, ERR_UNSUPPORTED = \
    -1, -2, -3, -4, -5, -6, -7
F64, F32 = 0, 1
PREC_F64, PREC_MIXED, PREC_MIXED_BF16 = 0, 1, 2
SOLVER_FCG, SOLVER_PCG, SOLVER_FGMRES = 0, 1, 2
COEF_CONSTANT, COEF_RADIAL_STEP = 0, 1
COEF_KINDS = {"diffusion": 0, "mass": 1}
COEF_WHERE = {"element": 0, "node": 1, "analytic": 2}
SMOOTHERS = {"none": 0, "point": 1, "block": 2, "schwarz": 3}
TIMING_KINDS = {"apply": 0, "block": 1, "smooth": 2, "schwarz": 3}
RHS_IDS = {"sinsinsin": 0, "shell_harmonic": 1, "radial_step": 2, "polynomial": 3, "gaussians": 4,
           "polynomial_dirichlet": 5, "star": 6}
NL_IDS = {"puncture": 0, "nl_quadratic": 1, "star": 2}

EXPORTED = ["hpdg_create", "hpdg_destroy", "hpdg_last_error", "hpdg_mesh_upload", "hpdg_mesh_info_get",
            "hpdg_level_cells", "hpdg_mesh_free", "hpdg_assemble_rhs", "hpdg_apply",
            "hpdg_setup_smoother", "hpdg_smooth", "hpdg_vcycle", "hpdg_solve",
            "hpdg_nonlinear_residual", "hpdg_nonlinear_linearize", "hpdg_newton_solve",
            "hpdg_server_create", "hpdg_server_submit", "hpdg_server_poll", "hpdg_server_wait",
            "hpdg_server_destroy", "hpdg_timing_enable", "hpdg_kernel_timing", "hpdg_apply_noalloc",
            "hpdg_set_coefficient", "hpdg_estimate", "hpdg_amr_mark", "hpdg_amr_smooth_pred",
            "hpdg_amr_adapt", "hpdg_transfer", "hpdg_set_estimator_grid"]


class HpdgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("hpdg error %d: %s" % (code, msg))
        self.code = code


class MeshDesc(ctypes.Structure):
    _fields_ = [("n_macro", ctypes.c_int32), ("macro_kind", ctypes.c_void_p),
                ("macro_params", ctypes.c_void_p), ("macro_nbr", ctypes.c_void_p),
                ("macro_nbr_face", ctypes.c_void_p), ("macro_nbr_orient", ctypes.c_void_p),
                ("macro_bc", ctypes.c_void_p), ("n_elem", ctypes.c_int64),
                ("elem_macro", ctypes.c_void_p), ("elem_level", ctypes.c_void_p),
                ("elem_anchor", ctypes.c_void_p), ("elem_p", ctypes.c_void_p)]


class DiscParams(ctypes.Structure):
    _fields_ = [("penalty_C", ctypes.c_double), ("quad_extra", ctypes.c_int32),
                ("coef_kind", ctypes.c_int32), ("coef_params", ctypes.c_double * 4),
                ("max_levels", ctypes.c_int32), ("build_f32", ctypes.c_int32), ("mass_term", ctypes.c_int32),
                ("robin_gamma", ctypes.c_double), ("ec_mode", ctypes.c_int32)]


class MeshInfo(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int32), ("n_elem", ctypes.c_int64 * 32),
                ("n_dof", ctypes.c_int64 * 32), ("n_mortar", ctypes.c_int64 * 32),
                ("vgeo_scalars", ctypes.c_int64 * 32), ("mgeo_scalars", ctypes.c_int64 * 32),
                ("table_bytes", ctypes.c_int64 * 32), ("device_bytes", ctypes.c_size_t),
                ("block_retries", ctypes.c_int32), ("coarse_retries", ctypes.c_int32),
                ("n_elem_centric", ctypes.c_int64 * 32), ("n_mortar_tasks", ctypes.c_int64 * 32),
                ("apply_flops", ctypes.c_double * 32), ("est_alg_bytes", ctypes.c_int64),
                ("est_volume_points", ctypes.c_int64), ("est_mortar_points", ctypes.c_int64)]


class SmootherParams(ctypes.Structure):
    _fields_ = [("n_cheb", ctypes.c_int32), ("n_eigs", ctypes.c_int32), ("Lambda", ctypes.c_double),
                ("scaling", ctypes.c_int32), ("seed", ctypes.c_uint64), ("n_cheb_coarse", ctypes.c_int32),
                ("unfused", ctypes.c_int32), ("schwarz_overlap", ctypes.c_int32)]


class SolveParams(ctypes.Structure):
    _fields_ = [("solver", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("tol_rel", ctypes.c_double), ("max_iter", ctypes.c_int32), ("restart", ctypes.c_int32)]


class SolveStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("rel_residual", ctypes.c_double),
                ("solve_ms", ctypes.c_double), ("status", ctypes.c_int32)]


class RhsDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_params", ctypes.c_int32), ("params", ctypes.c_void_p)]


class ServerParams(ctypes.Structure):
    _fields_ = [("max_active", ctypes.c_int32), ("hbm_budget_bytes", ctypes.c_size_t), ("precision", ctypes.c_int32),
                ("smoother", SmootherParams), ("tol_rel", ctypes.c_double), ("max_iter", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("mesh", MeshDesc), ("disc", DiscParams), ("rhs", RhsDesc), ("u_out", ctypes.c_void_p)]


class RequestStatus(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("status", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("rel_residual", ctypes.c_double), ("submit_ms", ctypes.c_double), ("start_ms", ctypes.c_double),
                ("end_ms", ctypes.c_double), ("device_bytes", ctypes.c_size_t), ("n_dof", ctypes.c_int64),
                ("message", ctypes.c_char * 200)]


class NonlinearDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_params", ctypes.c_int32), ("params", ctypes.c_void_p)]


class NewtonParams(ctypes.Structure):
    _fields_ = [("tol_rel", ctypes.c_double), ("lin_tol_rel", ctypes.c_double), ("max_newton", ctypes.c_int32),
                ("max_lin_iter", ctypes.c_int32), ("precision", ctypes.c_int32)]


class NewtonStats(ctypes.Structure):
    _fields_ = [("newton_steps", ctypes.c_int32), ("linear_iterations", ctypes.c_int32),
                ("rel_residual", ctypes.c_double), ("solve_ms", ctypes.c_double), ("status", ctypes.c_int32)]


_lib = None
# (block, coarse) setup retries of every mesh freed through Mesh.free(), for callers that check
# that no factorisation had to be repeated
RETRY_LOG = []


def load_library(path=LIB_PATH):
    """Load libhpdg.so; raises when it is missing (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libhpdg.so not built: run `python -m paper_1907_01572_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
    lib.hpdg_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.c_size_t]
    lib.hpdg_destroy.argtypes = [vp]
    lib.hpdg_last_error.argtypes = [vp]
    lib.hpdg_last_error.restype = ctypes.c_char_p
    lib.hpdg_mesh_upload.argtypes = [vp, ctypes.POINTER(MeshDesc), ctypes.POINTER(DiscParams),
                                     ctypes.POINTER(vp), vp]
    lib.hpdg_mesh_info_get.argtypes = [vp, ctypes.POINTER(MeshInfo)]
    lib.hpdg_level_cells.argtypes = [vp, i32, vp, vp, vp, vp]
    lib.hpdg_mesh_free.argtypes = [vp]
    lib.hpdg_assemble_rhs.argtypes = [vp, ctypes.POINTER(RhsDesc), vp, vp]
    lib.hpdg_apply.argtypes = [vp, i32, i32, vp, vp, vp]
    lib.hpdg_apply_noalloc.argtypes = [vp, i32, i32, vp, vp, vp]
    lib.hpdg_set_coefficient.argtypes = [vp, i32, i32, vp, vp, vp]
    lib.hpdg_estimate.argtypes = [vp, ctypes.POINTER(RhsDesc), vp, vp, vp, vp]
    lib.hpdg_amr_mark.argtypes = [vp, i64, i32, ctypes.c_double, vp]
    lib.hpdg_amr_smooth_pred.argtypes = [vp, vp, vp, vp, i64, ctypes.c_double, ctypes.c_double, vp, vp]
    lib.hpdg_amr_adapt.argtypes = [ctypes.POINTER(MeshDesc), vp, i32, i64, vp, vp, vp, vp, vp, vp]
    lib.hpdg_transfer.argtypes = [vp, vp, vp, vp, vp]
    lib.hpdg_set_estimator_grid.argtypes = [vp, ctypes.POINTER(MeshDesc)]
    lib.hpdg_setup_smoother.argtypes = [vp, ctypes.POINTER(SmootherParams), vp, vp]
    lib.hpdg_smooth.argtypes = [vp, i32, i32, vp, vp, i32, vp]
    lib.hpdg_vcycle.argtypes = [vp, i32, vp, vp, vp]
    lib.hpdg_solve.argtypes = [vp, ctypes.POINTER(SolveParams), vp, vp, ctypes.POINTER(SolveStats), vp]
    lib.hpdg_nonlinear_residual.argtypes = [vp, ctypes.POINTER(NonlinearDesc), vp, vp, vp, vp]
    lib.hpdg_nonlinear_linearize.argtypes = [vp, ctypes.POINTER(NonlinearDesc), vp, vp]
    lib.hpdg_newton_solve.argtypes = [vp, ctypes.POINTER(NewtonParams), ctypes.POINTER(NonlinearDesc), vp, vp,
                                      ctypes.POINTER(NewtonStats), vp]
    lib.hpdg_server_create.argtypes = [vp, ctypes.POINTER(ServerParams), ctypes.POINTER(vp)]
    lib.hpdg_server_submit.argtypes = [vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
    lib.hpdg_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(RequestStatus)]
    lib.hpdg_server_wait.argtypes = [vp, ctypes.c_uint64, i64, ctypes.POINTER(RequestStatus)]
    lib.hpdg_server_destroy.argtypes = [vp]
    lib.hpdg_timing_enable.argtypes = [vp, i32]
    lib.hpdg_kernel_timing.argtypes = [vp, i32, i32, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64),
                                       ctypes.POINTER(ctypes.c_double)]
    _lib = lib
    return lib


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Context:
    """One library context on a HIP device (all device memory of its meshes)."""

    def __init__(self, device=0, hbm_budget_bytes=0):
        self.lib = load_library()
        self.h = ctypes.c_void_p()
        rc = self.lib.hpdg_create(ctypes.byref(self.h), int(device), int(hbm_budget_bytes))
        if rc != OK:
            raise HpdgError(rc, "hpdg_create failed")
        self.meshes = []

    def check(self, rc):
        if rc != OK:
            raise HpdgError(rc, self.lib.hpdg_last_error(self.h).decode())
        return rc

    def upload(self, mesh, penalty_C=10.0, quad_extra=1, coef=None, max_levels=0, build_f32=False,
               stream=None, mass_term=False, robin_gamma=0.0, ec_mode=None):
        """``mass_term``: levels carry the Newton mass form (needed by the nonlinear calls);
        ``robin_gamma``: gamma of the Robin faces (macro face kind 3); ``ec_mode``: EC_AUTO,
        EC_ALWAYS or EC_NEVER (None: EC_MODE_DEFAULT)."""
        return Mesh(self, mesh, penalty_C, quad_extra, coef, max_levels, build_f32, stream, mass_term, robin_gamma,
                    ec_mode)

    def close(self):
        if self.h:
            for m in list(self.meshes):
                m.h = None
            self.lib.hpdg_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def coef_from_problem(problem):
    """Coefficient descriptor (kind, params) of a meshgen problem."""
    if problem is not None and problem.get("kind") == "radial_step":
        return COEF_RADIAL_STEP, list(problem["params"][:3]) + [0.0]
    return COEF_CONSTANT, [0.0] * 4


# element-centric apply (hpdg_disc_params.ec_mode): by level, always, never
EC_AUTO, EC_ALWAYS, EC_NEVER = 0, 1, 2
# the mode of uploads that do not name one
EC_MODE_DEFAULT = EC_AUTO


def _descriptors(mesh, penalty_C=10.0, quad_extra=1, coef=None, max_levels=0, build_f32=False, mass_term=False,
                 robin_gamma=0.0, ec_mode=None):
    """C descriptors of a meshgen mesh; returns (MeshDesc, DiscParams, arrays to keep alive)."""
    keep = dict(
        macro_kind=np.ascontiguousarray(mesh["macro_kind"], np.int32),
        macro_params=np.ascontiguousarray(mesh["macro_params"], np.float64),
        macro_nbr=np.ascontiguousarray(mesh["macro_nbr"], np.int32),
        macro_nbr_face=np.ascontiguousarray(mesh["macro_nbr_face"], np.int32),
        macro_nbr_orient=np.ascontiguousarray(mesh["macro_nbr_orient"], np.int32),
        macro_bc=np.ascontiguousarray(mesh["macro_bc"], np.int32),
        elem_macro=np.ascontiguousarray(mesh["elem_macro"], np.int32),
        elem_level=np.ascontiguousarray(mesh["elem_level"], np.int32),
        elem_anchor=np.ascontiguousarray(mesh["elem_anchor"], np.int32),
        elem_p=np.ascontiguousarray(mesh["elem_p"], np.int32))
    d = MeshDesc()
    d.n_macro = len(keep["macro_kind"])
    d.n_elem = len(keep["elem_p"])
    for k, v in keep.items():
        setattr(d, k, v.ctypes.data)
    dp = DiscParams()
    dp.penalty_C = penalty_C
    dp.quad_extra = quad_extra
    kind, params = coef if coef is not None else (COEF_CONSTANT, [0.0] * 4)
    dp.coef_kind = kind
    for i in range(4):
        dp.coef_params[i] = params[i]
    dp.max_levels = max_levels
    dp.build_f32 = 1 if build_f32 else 0
    dp.mass_term = 1 if mass_term else 0
    dp.robin_gamma = robin_gamma
    dp.ec_mode = EC_MODE_DEFAULT if ec_mode is None else ec_mode
    return d, dp, keep


# hp-adaptation (host steps of the library; no context needed)
MARK_FRACTION, MARK_MEAN = 0, 1


def _host_check(lib, rc):
    if rc != OK:
        raise HpdgError(rc, lib.hpdg_last_error(None).decode())


def amr_mark(eta2, mode, param):
    """Marked elements (bool array) of eta2: MARK_FRACTION (largest ceil(param E)) or MARK_MEAN
    (eta2 > param * mean)."""
    lib = load_library()
    e = np.ascontiguousarray(eta2, np.float64)
    out = np.zeros(len(e), np.uint8)
    _host_check(lib, lib.hpdg_amr_mark(e.ctypes.data, len(e), int(mode), float(param), out.ctypes.data))
    return out.astype(bool)


def amr_smooth_pred(eta2, eta2_pred, p, marked, gamma_h=0.25, gamma_p=0.1):
    """(action, prediction) per element: 0 keep, 1 h-refine, 2 p-refine; eta2_pred = inf means
    no prediction."""
    lib = load_library()
    e = np.ascontiguousarray(eta2, np.float64)
    pr = np.ascontiguousarray(eta2_pred, np.float64)
    pp = np.ascontiguousarray(p, np.int32)
    mk = np.ascontiguousarray(marked, np.uint8)
    act = np.zeros(len(e), np.int8)
    out = np.zeros(len(e), np.float64)
    _host_check(lib, lib.hpdg_amr_smooth_pred(e.ctypes.data, pr.ctypes.data, pp.ctypes.data, mk.ctypes.data,
                                              len(e), float(gamma_h), float(gamma_p), act.ctypes.data,
                                              out.ctypes.data))
    return act, out


def amr_adapt(mesh, action, max_degree=15):
    """(new mesh, origin): ``mesh`` (a meshgen mesh dict) with action[e] applied and 2:1 balance
    restored; origin[i] = the old cell of new cell i."""
    lib = load_library()
    d, _, keep = _descriptors(mesh)
    act = np.ascontiguousarray(action, np.int8)
    if len(act) != d.n_elem:
        raise ValueError("one action per element")
    cap = 8 * d.n_elem
    macro, level, p = (np.zeros(cap, np.int32) for _ in range(3))
    anchor = np.zeros((cap, 3), np.int32)
    origin = np.zeros(cap, np.int64)
    n = ctypes.c_int64()
    _host_check(lib, lib.hpdg_amr_adapt(ctypes.byref(d), act.ctypes.data, int(max_degree), cap, macro.ctypes.data,
                                        level.ctypes.data, anchor.ctypes.data, p.ctypes.data, origin.ctypes.data,
                                        ctypes.byref(n)))
    k = n.value
    out = dict(mesh)
    out.update(elem_macro=macro[:k].copy(), elem_level=level[:k].copy(), elem_anchor=anchor[:k].copy(),
               elem_p=p[:k].copy())
    return out, origin[:k].copy()


REQ_STATES = {0: "queued", 1: "running", 2: "done", 3: "failed"}


class Server:
    """Continuous-batching solve server (hpdg_server_*): independent linear solves admitted
    by device footprint, ``max_active`` in flight on their own streams."""

    def __init__(self, ctx, max_active=4, hbm_budget_bytes=0, precision=PREC_F64, n_cheb=4, Lambda=20.0,
                 n_eigs=15, smoother="point", seed=0, tol=1e-10, max_iter=1000):
        self.ctx, self.lib = ctx, ctx.lib
        sp = SmootherParams(n_cheb, n_eigs, Lambda, SMOOTHERS[smoother], seed, 0, 0, 2)
        p = ServerParams(max_active, hbm_budget_bytes, precision, sp, tol, max_iter)
        self.h = ctypes.c_void_p()
        ctx.check(self.lib.hpdg_server_create(ctx.h, ctypes.byref(p), ctypes.byref(self.h)))
        self._keep = {}

    def submit(self, mesh, problem, out, coef=None):
        """Queue a solve of the mesh with the problem's RHS; ``out`` (float64 numpy array of
        the mesh's DOF count) receives the solution.  Returns the ticket."""
        assert out.dtype == np.float64 and out.flags["C_CONTIGUOUS"]
        d, dp, keep = _descriptors(mesh, coef=coef if coef is not None else coef_from_problem(problem))
        params = np.ascontiguousarray(problem["params"], np.float64).reshape(-1)
        r = Request()
        r.mesh = d
        r.disc = dp
        r.rhs.kind = RHS_IDS[problem["kind"]]
        r.rhs.n_params = len(params)
        r.rhs.params = params.ctypes.data if len(params) else None
        r.u_out = out.ctypes.data
        t = ctypes.c_uint64()
        self.ctx.check(self.lib.hpdg_server_submit(self.h, ctypes.byref(r), ctypes.byref(t)))
        self._keep[t.value] = out  # the descriptors were copied; the output buffer must stay alive
        return t.value

    @staticmethod
    def _status(st):
        return dict(state=REQ_STATES[st.state], status=st.status, iterations=st.iterations,
                    rel_residual=st.rel_residual, submit_ms=st.submit_ms, start_ms=st.start_ms,
                    end_ms=st.end_ms, device_bytes=int(st.device_bytes), n_dof=int(st.n_dof),
                    message=st.message.decode(errors="replace"))

    def poll(self, ticket):
        st = RequestStatus()
        self.ctx.check(self.lib.hpdg_server_poll(self.h, ticket, ctypes.byref(st)))
        return self._status(st)

    def wait(self, ticket, timeout_ms=-1):
        st = RequestStatus()
        self.ctx.check(self.lib.hpdg_server_wait(self.h, ticket, int(timeout_ms), ctypes.byref(st)))
        out = self._status(st)
        if out["state"] in ("done", "failed"):
            self._keep.pop(ticket, None)
        return out

    def close(self):
        if self.h:
            self.lib.hpdg_server_destroy(self.h)
            self.h = None
            self._keep.clear()


class Mesh:
    """An uploaded mesh: level hierarchy, geometry and solver state on the device."""

    def __init__(self, ctx, mesh, penalty_C, quad_extra, coef, max_levels, build_f32, stream, mass_term=False,
                 robin_gamma=0.0, ec_mode=None):
        self.ctx, self.lib = ctx, ctx.lib
        d, dp, self._keep = _descriptors(mesh, penalty_C, quad_extra, coef, max_levels, build_f32, mass_term,
                                         robin_gamma, ec_mode)
        self.h = ctypes.c_void_p()
        ctx.check(self.lib.hpdg_mesh_upload(ctx.h, ctypes.byref(d), ctypes.byref(dp),
                                            ctypes.byref(self.h), _stream(stream)))
        self._after_upload()

    def _after_upload(self):
        ctx = self.ctx
        ctx.meshes.append(self)
        info = MeshInfo()
        ctx.check(self.lib.hpdg_mesh_info_get(self.h, ctypes.byref(info)))
        self.n_levels = info.n_levels
        self.n_dof = [int(info.n_dof[i]) for i in range(self.n_levels)]
        self.n_elem = [int(info.n_elem[i]) for i in range(self.n_levels)]
        self.n_mortar = [int(info.n_mortar[i]) for i in range(self.n_levels)]
        self.vgeo_scalars = [int(info.vgeo_scalars[i]) for i in range(self.n_levels)]
        self.mgeo_scalars = [int(info.mgeo_scalars[i]) for i in range(self.n_levels)]
        self.table_bytes = [int(info.table_bytes[i]) for i in range(self.n_levels)]
        self.device_bytes = int(info.device_bytes)
        self.block_retries = int(info.block_retries)
        self.coarse_retries = int(info.coarse_retries)
        self.n_elem_centric = [int(info.n_elem_centric[i]) for i in range(self.n_levels)]
        self.n_mortar_tasks = [int(info.n_mortar_tasks[i]) for i in range(self.n_levels)]
        self.apply_flops = [float(info.apply_flops[i]) for i in range(self.n_levels)]

    def algorithmic_bytes(self, level=0, scalar=8):
        """Bytes one apply of ``level`` must move at least once: x read and y written, the
        stored volume and mortar metric, and the element / mortar records."""
        return (2 * scalar * self.n_dof[level] + scalar * (self.vgeo_scalars[level] + self.mgeo_scalars[level])
                + self.table_bytes[level])

    def level_cells(self, level):
        E = self.n_elem[level]
        macro, lvl, p = (np.zeros(E, np.int32) for _ in range(3))
        anchor = np.zeros((E, 3), np.int32)
        self.ctx.check(self.lib.hpdg_level_cells(self.h, level, macro.ctypes.data, lvl.ctypes.data,
                                                 anchor.ctypes.data, p.ctypes.data))
        return dict(elem_macro=macro, elem_level=lvl, elem_anchor=anchor, elem_p=p)

    def assemble_rhs(self, problem, F, stream=None):
        params = np.ascontiguousarray(problem["params"], np.float64).reshape(-1)
        r = RhsDesc()
        r.kind = RHS_IDS[problem["kind"]]
        r.n_params = len(params)
        r.params = params.ctypes.data if len(params) else None
        self.ctx.check(self.lib.hpdg_assemble_rhs(self.h, ctypes.byref(r), _ptr(F), _stream(stream)))

    def estimate(self, problem, u, eta2, eta2_vol=None, stream=None):
        """eta2[e] (FP64 device tensor of n_elem[0]): the a posteriori estimate of the level-0
        vector u for ``problem``; eta2_vol (optional): its volume parts."""
        params = np.ascontiguousarray(problem["params"], np.float64).reshape(-1)
        r = RhsDesc()
        r.kind = RHS_IDS[problem["kind"]]
        r.n_params = len(params)
        r.params = params.ctypes.data if len(params) else None
        self.ctx.check(self.lib.hpdg_estimate(self.h, ctypes.byref(r), _ptr(u), _ptr(eta2),
                                              _ptr(eta2_vol) if eta2_vol is not None else None,
                                              _stream(stream)))


    def set_estimator_grid(self, grid=None):
        """The fiducial grid of the estimator: a mesh dict with this mesh's macro connectivity
        (its macro maps are used); None: the physical grid."""
        if grid is None:
            self.ctx.check(self.lib.hpdg_set_estimator_grid(self.h, None))
            return
        d, _, keep = _descriptors(grid)
        self.ctx.check(self.lib.hpdg_set_estimator_grid(self.h, ctypes.byref(d)))

    def estimate_info(self):
        """(algorithmic bytes, volume points, mortar points) of one estimate of the last problem
        estimated (zeros before the first)."""
        info = MeshInfo()
        self.ctx.check(self.lib.hpdg_mesh_info_get(self.h, ctypes.byref(info)))
        return int(info.est_alg_bytes), int(info.est_volume_points), int(info.est_mortar_points)

    def transfer_to(self, other, u, u_other, stream=None):
        """u_other (level-0 vector of ``other``, an adapted copy of this mesh) = u carried over."""
        self.ctx.check(self.lib.hpdg_transfer(self.h, other.h, _ptr(u), _ptr(u_other), _stream(stream)))

    def apply(self, x, y, level=0, stream=None):
        prec = F32 if x.dtype.itemsize == 4 else F64
        self.ctx.check(self.lib.hpdg_apply(self.h, level, prec, _ptr(x), _ptr(y), _stream(stream)))

    def set_coefficient(self, kind, where, values=None, params=None, stream=None):
        """k ("diffusion") or c ("mass") per "element" (values[n_elem[0]]), per "node" (values[n_dof[0]],
        level-vector layout) or "analytic" (params); rebuilds the level tables (and the smoother)."""
        vals = None if values is None else np.ascontiguousarray(values, np.float64)
        par = None if params is None else np.ascontiguousarray(params, np.float64)
        self.ctx.check(self.lib.hpdg_set_coefficient(self.h, COEF_KINDS[kind], COEF_WHERE[where],
                                                     vals.ctypes.data if vals is not None else None,
                                                     par.ctypes.data if par is not None else None,
                                                     _stream(stream)))
        self._after_info()

    def _after_info(self):
        info = MeshInfo()
        self.ctx.check(self.lib.hpdg_mesh_info_get(self.h, ctypes.byref(info)))
        self.vgeo_scalars = [int(info.vgeo_scalars[i]) for i in range(self.n_levels)]
        self.mgeo_scalars = [int(info.mgeo_scalars[i]) for i in range(self.n_levels)]
        self.table_bytes = [int(info.table_bytes[i]) for i in range(self.n_levels)]
        self.device_bytes = int(info.device_bytes)

    def apply_noalloc(self, x, y, level=0, stream=None):
        """y = A x with the face traces in the library's fixed scratch (no device allocation)."""
        prec = F32 if x.dtype.itemsize == 4 else F64
        self.ctx.check(self.lib.hpdg_apply_noalloc(self.h, level, prec, _ptr(x), _ptr(y), _stream(stream)))

    def setup_smoother(self, n_cheb=4, n_eigs=15, Lambda=20.0, jacobi=True, seed=0, lambda_max=None,
                       smoother=None, stream=None, n_cheb_coarse=0, fused=True, schwarz_overlap=2):
        """``smoother``: "none", "point", "block" (Chebyshev) or "schwarz" (additive Schwarz
        with ``n_cheb`` cycles per call and ``schwarz_overlap`` = N_overlap; FP64, and FP32 on meshes with FP32 levels)
        (default: "point" if jacobi else "none").
        ``n_cheb_coarse``: Chebyshev steps (Schwarz cycles) on the levels below the finest (0: ``n_cheb``).
        ``fused``: block smoothing on one-degree levels runs the apply and the block step as one
        kernel (False: separate kernels)."""
        kind = smoother if smoother is not None else ("point" if jacobi else "none")
        sp = SmootherParams(n_cheb, n_eigs, Lambda, SMOOTHERS[kind], seed, n_cheb_coarse, 0 if fused else 1,
                            schwarz_overlap)
        lam = np.zeros(max(self.n_levels - 1, 1))
        if lambda_max is not None:
            lam[:len(lambda_max)] = lambda_max
        self.ctx.check(self.lib.hpdg_setup_smoother(self.h, ctypes.byref(sp), lam.ctypes.data,
                                                    _stream(stream)))
        self.lambda_max = lam[: self.n_levels - 1].copy()
        return self.lambda_max

    def smooth(self, b, x, level=0, n_iter=4, stream=None):
        prec = F32 if b.dtype.itemsize == 4 else F64
        self.ctx.check(self.lib.hpdg_smooth(self.h, level, prec, _ptr(b), _ptr(x), n_iter, _stream(stream)))

    def vcycle(self, r, z, stream=None):
        prec = F32 if r.dtype.itemsize == 4 else F64
        self.ctx.check(self.lib.hpdg_vcycle(self.h, prec, _ptr(r), _ptr(z), _stream(stream)))

    def solve(self, b, u, tol=1e-10, max_iter=200, solver=SOLVER_FCG, precision=PREC_F64, stream=None,
              raise_on_error=True, restart=0):
        p = SolveParams(solver, precision, tol, max_iter, restart)
        st = SolveStats()
        rc = self.lib.hpdg_solve(self.h, ctypes.byref(p), _ptr(b), _ptr(u), ctypes.byref(st), _stream(stream))
        if raise_on_error:
            self.ctx.check(rc)
        return dict(iterations=st.iterations, rel_residual=st.rel_residual, solve_ms=st.solve_ms,
                    status=st.status)

    def _nl(self, nl):
        params = np.ascontiguousarray(nl["params"], np.float64).reshape(-1)
        d = NonlinearDesc()
        d.kind = NL_IDS[nl["kind"]]
        d.n_params = len(params)
        d.params = params.ctypes.data
        return d, params

    def nonlinear_residual(self, nl, u, R, F=None, stream=None):
        """R = A u - N(u) - F (F None: zero)."""
        d, keep = self._nl(nl)
        self.ctx.check(self.lib.hpdg_nonlinear_residual(self.h, ctypes.byref(d), _ptr(F) if F is not None else None,
                                                        _ptr(u), _ptr(R), _stream(stream)))

    def linearize(self, nl, u, stream=None):
        """Set every level's Jacobian mass term from u; afterwards ``apply`` applies J."""
        d, keep = self._nl(nl)
        self.ctx.check(self.lib.hpdg_nonlinear_linearize(self.h, ctypes.byref(d), _ptr(u), _stream(stream)))

    def newton_solve(self, nl, u, F=None, tol=1e-10, lin_tol=1e-6, max_newton=30, max_lin_iter=500,
                     precision=PREC_F64, stream=None, raise_on_error=True):
        d, keep = self._nl(nl)
        p = NewtonParams(tol, lin_tol, max_newton, max_lin_iter, precision)
        st = NewtonStats()
        rc = self.lib.hpdg_newton_solve(self.h, ctypes.byref(p), ctypes.byref(d),
                                        _ptr(F) if F is not None else None, _ptr(u), ctypes.byref(st),
                                        _stream(stream))
        if raise_on_error:
            self.ctx.check(rc)
        return dict(newton_steps=st.newton_steps, linear_iterations=st.linear_iterations,
                    rel_residual=st.rel_residual, solve_ms=st.solve_ms, status=st.status)

    def timing_enable(self, every=1):
        """Time every ``every``-th launch of each kernel kind / level / precision (0: off)."""
        self.ctx.check(self.lib.hpdg_timing_enable(self.h, int(every)))

    def kernel_timing(self, kind="apply", level=0, prec=F64):
        """(total ms, launches, algorithmic bytes) recorded for one kernel kind, level and
        precision since the previous read of that entry; the entry is then reset."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        b = ctypes.c_double()
        k = TIMING_KINDS[kind]
        self.ctx.check(self.lib.hpdg_kernel_timing(self.h, k, level, prec, ctypes.byref(ms), ctypes.byref(n),
                                                   ctypes.byref(b)))
        return ms.value, n.value, b.value

    def setup_retries(self):
        """(block, coarse) setup factorisations repeated after a failed attempt (0, 0 when healthy)."""
        info = MeshInfo()
        self.ctx.check(self.lib.hpdg_mesh_info_get(self.h, ctypes.byref(info)))
        return int(info.block_retries), int(info.coarse_retries)

    def free(self):
        if self.h:
            RETRY_LOG.append(self.setup_retries())
            self.lib.hpdg_mesh_free(self.h)
            self.h = None
            if self in self.ctx.meshes:
                self.ctx.meshes.remove(self)
