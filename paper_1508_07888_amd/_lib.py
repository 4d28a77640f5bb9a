"""ctypes binding of libemma_rt.so (include/emma_rt.h), same names as the C ABI.

Argument marshalling only: every step of the radiation path runs in the HIP
kernels of the library.  Loading fails loudly when the library is not built.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libemma_rt.so")

MAX_GROUPS = 4
SUBSTEP_BINS = 18  # EMMA_RT_SUBSTEP_BINS
MAX_SOURCES = 65536

EMMA_RT_OK = 0
EMMA_RT_EINVAL = -1
EMMA_RT_ENOMEM = -2
EMMA_RT_EHIP = -3
EMMA_RT_ESUBSTEP = -4
EMMA_RT_ENONFINITE = -5
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ESUBSTEP", -5: "ENONFINITE"}

EMMA_RT_FP64 = 0
EMMA_RT_MIXED = 1
PATHS = {"split": 0, "fused": 1, "reference": 2}
BCS = {"periodic": 0, "transmissive": 1, "reflective": 2, "inflow": 3}
FLUXES = {"glf": 0, "hll": 1}

EXPORTS = ("emma_rt_init", "emma_rt_step", "emma_rt_step_crta", "emma_rt_step_adjoint", "emma_rt_free",
           "emma_rt_last_error", "emma_rt_group_constants", "emma_rt_scratch_bytes",
           "emma_rt_profile_enable", "emma_rt_profile_read", "emma_rt_step_noalloc",
           "emma_rt_step_crta_adjoint", "emma_rt_crta_adjoint_work_bytes")
NOALLOC_SCRATCH_BYTES = 128 << 20  # EMMA_RT_NOALLOC_SCRATCH_BYTES


class emma_rt_config(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("n_groups", ctypes.c_int32),
        ("dx", ctypes.c_double), ("c_red", ctypes.c_double),
        ("precision", ctypes.c_int32), ("otsa", ctypes.c_int32), ("isothermal", ctypes.c_int32),
        ("max_substeps", ctypes.c_int32), ("adjoint_max_steps", ctypes.c_int32),
        ("path", ctypes.c_int32),
        ("sigma_N", ctypes.c_double * MAX_GROUPS), ("sigma_E", ctypes.c_double * MAX_GROUPS),
        ("mean_E", ctypes.c_double * MAX_GROUPS), ("src_frac", ctypes.c_double * MAX_GROUPS),
        ("bc", ctypes.c_int32 * 6), ("flux", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("inflow", ctypes.c_double * 6),
    ]


class emma_rt_diag(ctypes.Structure):
    _fields_ = [
        ("photons", ctypes.c_double * MAX_GROUPS), ("ionised", ctypes.c_double),
        ("substeps", ctypes.c_int64), ("attempts", ctypes.c_int64),
        ("max_sub", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("limiter_hits", ctypes.c_int64), ("neg_clamps", ctypes.c_int64),
        ("x_clamps", ctypes.c_int64), ("cap_hits", ctypes.c_int64), ("nonfinite", ctypes.c_int64),
        ("substep_hist", ctypes.c_int64 * SUBSTEP_BINS),
    ]

    def as_dict(self, G):
        return {
            "photons": list(self.photons)[:G], "ionised": self.ionised,
            "substeps": self.substeps, "attempts": self.attempts, "max_sub": self.max_sub,
            "limiter_hits": self.limiter_hits, "neg_clamps": self.neg_clamps,
            "x_clamps": self.x_clamps, "cap_hits": self.cap_hits, "nonfinite": self.nonfinite,
            "substep_hist": list(self.substep_hist),
        }


class emma_rt_kernel_time(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double)]


_lib = None
_vp = ctypes.c_void_p


def load():
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -m paper_1508_07888_amd.build); there is no fallback path")
    L = ctypes.CDLL(LIB_PATH)
    L.emma_rt_init.restype = ctypes.c_int
    L.emma_rt_init.argtypes = [ctypes.POINTER(_vp), ctypes.POINTER(emma_rt_config), _vp]
    L.emma_rt_step.restype = ctypes.c_int
    L.emma_rt_step.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_double,
                               ctypes.c_int32, ctypes.POINTER(emma_rt_diag)]
    L.emma_rt_step_crta.restype = ctypes.c_int
    L.emma_rt_step_crta.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_int32,
                                    ctypes.c_double, ctypes.c_int32, _vp, ctypes.c_int32, ctypes.c_int32,
                                    _vp, _vp, _vp, ctypes.POINTER(emma_rt_diag)]
    L.emma_rt_step_adjoint.restype = ctypes.c_int
    L.emma_rt_step_adjoint.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_int32,
                                       ctypes.c_double, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, _vp]
    L.emma_rt_step_crta_adjoint.restype = ctypes.c_int
    L.emma_rt_step_crta_adjoint.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_int32,
                                            ctypes.c_double, ctypes.c_int32, _vp, ctypes.c_int32,
                                            ctypes.c_int32, _vp, _vp, _vp, _vp, ctypes.c_int64] + [_vp] * 9
    L.emma_rt_crta_adjoint_work_bytes.restype = ctypes.c_int64
    L.emma_rt_crta_adjoint_work_bytes.argtypes = [ctypes.c_int32] * 3
    L.emma_rt_free.restype = None
    L.emma_rt_free.argtypes = [_vp]
    L.emma_rt_last_error.restype = ctypes.c_char_p
    L.emma_rt_last_error.argtypes = [_vp]
    L.emma_rt_group_constants.restype = ctypes.c_int
    L.emma_rt_group_constants.argtypes = [ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                          ctypes.c_int32] + [ctypes.POINTER(ctypes.c_double)] * 4
    L.emma_rt_profile_enable.restype = ctypes.c_int
    L.emma_rt_profile_enable.argtypes = [_vp, ctypes.c_int32]
    L.emma_rt_profile_read.restype = ctypes.c_int
    L.emma_rt_profile_read.argtypes = [_vp, ctypes.POINTER(emma_rt_kernel_time), ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_int32)]
    L.emma_rt_step_noalloc.restype = ctypes.c_int
    L.emma_rt_step_noalloc.argtypes = [ctypes.POINTER(emma_rt_config), _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                       ctypes.c_int32, ctypes.c_double, ctypes.c_int32]
    L.emma_rt_scratch_bytes.restype = ctypes.c_int64
    L.emma_rt_scratch_bytes.argtypes = [ctypes.POINTER(emma_rt_config)]
    _lib = L
    return L


class EmmaError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.message = message


def emma_rt_group_constants(T_bb, edges_eV):
    L = load()
    G = len(edges_eV) - 1
    e = (ctypes.c_double * (G + 1))(*edges_eV)
    outs = [(ctypes.c_double * max(G, 1))() for _ in range(4)]
    rc = L.emma_rt_group_constants(float(T_bb), e, G, *outs)
    if rc != EMMA_RT_OK:
        raise EmmaError(rc, "bad group constants request")
    names = ("sigma_N", "sigma_E", "mean_E", "frac")
    return {k: [o[i] for i in range(G)] for k, o in zip(names, outs)}


def emma_rt_init(cfg, stream_ptr):
    L = load()
    ctx = _vp()
    rc = L.emma_rt_init(ctypes.byref(ctx), ctypes.byref(cfg), _vp(stream_ptr))
    if rc != EMMA_RT_OK:
        raise EmmaError(rc, L.emma_rt_last_error(None).decode())
    return ctx


def emma_rt_step_crta(ctx, N, F, x, T, n0, src_cell, src_rate, src_child, n_src, dt, n_steps, ref_cell, n_ref,
                      ratio, x_fine, T_fine, n_fine, diag=None):
    """Pointers are integers (device addresses, 0 = NULL); returns the status code."""
    L = load()
    return L.emma_rt_step_crta(ctx, _vp(N), _vp(F), _vp(x), _vp(T), _vp(n0), _vp(src_cell), _vp(src_rate),
                               _vp(src_child), int(n_src), float(dt), int(n_steps), _vp(ref_cell), int(n_ref),
                               int(ratio), _vp(x_fine), _vp(T_fine), _vp(n_fine),
                               ctypes.byref(diag) if diag is not None else None)


def emma_rt_step(ctx, N, F, x, T, n0, src_cell, src_rate, n_src, dt, n_steps, diag=None):
    """Pointers are integers (device addresses); returns the status code."""
    L = load()
    return L.emma_rt_step(ctx, _vp(N), _vp(F), _vp(x), _vp(T), _vp(n0), _vp(src_cell),
                          _vp(src_rate), int(n_src), float(dt), int(n_steps),
                          ctypes.byref(diag) if diag is not None else None)


def emma_rt_step_noalloc(cfg, stream_ptr, N, F, x, T, n0, src_cell, src_rate, n_src, dt, n_steps):
    """emma_rt_step without a context or any allocation (fixed library scratch);
    pointers are integers (device addresses); returns the status code."""
    L = load()
    return L.emma_rt_step_noalloc(ctypes.byref(cfg), _vp(stream_ptr), _vp(N), _vp(F), _vp(x), _vp(T), _vp(n0),
                                  _vp(src_cell), _vp(src_rate), int(n_src), float(dt), int(n_steps))


def emma_rt_step_adjoint(ctx, N0, F0, x0, T0, n0, src_cell, src_rate, n_src, dt, n_steps,
                         gN, gF, gx, gT, g_n0, g_rate):
    L = load()
    return L.emma_rt_step_adjoint(ctx, _vp(N0), _vp(F0), _vp(x0), _vp(T0), _vp(n0), _vp(src_cell),
                                  _vp(src_rate), int(n_src), float(dt), int(n_steps), _vp(gN),
                                  _vp(gF), _vp(gx), _vp(gT), _vp(g_n0), _vp(g_rate))


def emma_rt_crta_adjoint_work_bytes(n_steps, n_ref, ratio):
    return load().emma_rt_crta_adjoint_work_bytes(int(n_steps), int(n_ref), int(ratio))


def emma_rt_step_crta_adjoint(ctx, N0, F0, x0, T0, n0, src_cell, src_rate, src_child, n_src, dt, n_steps,
                              ref_cell, n_ref, ratio, x_fine0, T_fine0, n_fine, work, work_bytes,
                              gN, gF, gx, gT, g_n0, g_rate, g_x_fine, g_T_fine, g_n_fine):
    """Pointers are integers (device addresses, 0 = NULL); returns the status code."""
    L = load()
    return L.emma_rt_step_crta_adjoint(ctx, _vp(N0), _vp(F0), _vp(x0), _vp(T0), _vp(n0), _vp(src_cell),
                                       _vp(src_rate), _vp(src_child), int(n_src), float(dt), int(n_steps),
                                       _vp(ref_cell), int(n_ref), int(ratio), _vp(x_fine0), _vp(T_fine0),
                                       _vp(n_fine), _vp(work), int(work_bytes), _vp(gN), _vp(gF), _vp(gx),
                                       _vp(gT), _vp(g_n0), _vp(g_rate), _vp(g_x_fine), _vp(g_T_fine),
                                       _vp(g_n_fine))


def emma_rt_free(ctx):
    if ctx:
        load().emma_rt_free(ctx)


def emma_rt_last_error(ctx):
    return load().emma_rt_last_error(ctx).decode()


def emma_rt_scratch_bytes(cfg):
    return load().emma_rt_scratch_bytes(ctypes.byref(cfg))


def emma_rt_profile_enable(ctx, enable):
    rc = load().emma_rt_profile_enable(ctx, int(bool(enable)))
    if rc != EMMA_RT_OK:
        raise EmmaError(rc, emma_rt_last_error(ctx))


def emma_rt_profile_read(ctx):
    """{kernel name: (launches, total ms)} since the last read."""
    out = (emma_rt_kernel_time * 16)()
    n = ctypes.c_int32(0)
    rc = load().emma_rt_profile_read(ctx, out, 16, ctypes.byref(n))
    if rc != EMMA_RT_OK:
        raise EmmaError(rc, emma_rt_last_error(ctx))
    return {out[i].name.decode(): (int(out[i].launches), float(out[i].total_ms))
            for i in range(n.value)}
