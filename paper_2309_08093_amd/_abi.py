"""ctypes declarations of the C ABI in include/tt_sketch.h (argument marshalling only)."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libttsketch.so")

TT_OK, TT_ERR_ARG, TT_ERR_SHAPE, TT_ERR_WORKSPACE, TT_ERR_HIP, TT_ERR_NOT_SPD, TT_ERR_NONFINITE, TT_ERR_STATE = range(8)
STATUS_NAMES = {0: "TT_OK", 1: "TT_ERR_ARG", 2: "TT_ERR_SHAPE", 3: "TT_ERR_WORKSPACE", 4: "TT_ERR_HIP",
                5: "TT_ERR_NOT_SPD", 6: "TT_ERR_NONFINITE", 7: "TT_ERR_STATE"}
TT_F64, TT_F32, TT_BF16 = 0, 1, 2
TT_GRAM_WORK, TT_GRAM_BF16 = 0, 1
TT_FLAG_SERIAL = 1
TT_FLAG_FUSE = 2
TT_FLAG_NO_FUSE = 4
TT_FLAG_EXACT = 8
TT_FLAG_INNER = 16
TT_FLAG_NO_INNER = 32

MAX_ORDER, MAX_J, MAX_RANK, MAX_S, MAX_N0 = 16, 8192, 16, 180, 4096
NOALLOC_SCRATCH_BYTES = 32 << 20


class PlanDesc(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int32),
        ("n", ctypes.POINTER(ctypes.c_int64)),
        ("r", ctypes.POINTER(ctypes.c_int64)),
        ("J", ctypes.c_int64),
        ("lambda_", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("x_dtype", ctypes.c_int32),
        ("work_dtype", ctypes.c_int32),
        ("gram_mode", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
    ]


_vp = ctypes.c_void_p
_vpp = ctypes.POINTER(ctypes.c_void_p)

# (name, argtypes) of every exported entry point; all return tt_status (int)
# except the two string getters.
SIGNATURES = {
    "tt_sketch_plan": [ctypes.POINTER(PlanDesc), _vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(_vp)],
    "tt_plan_bind_workspace": [_vp, _vp, ctypes.c_size_t],
    "tt_plan_set_stream": [_vp, _vp],
    "tt_plan_destroy": [_vp],
    "tt_plan_set_sweep": [_vp, ctypes.c_int64],
    "tt_plan_get_sweep": [_vp, ctypes.POINTER(ctypes.c_int64)],
    "tt_plan_get_tables": [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int8)],
    "tt_plan_set_tables": [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int8)],
    "tt_sketch_tensor": [_vp, _vp, ctypes.c_int32, _vp],
    "tt_sketch_tensor_all": [_vp, _vp, _vp],
    "tt_sketch_sparse": [_vp, ctypes.c_int64, _vp, _vp, ctypes.c_int32, _vp],
    "tt_sketch_sparse_all": [_vp, ctypes.c_int64, _vp, _vp, _vp],
    "tt_exact_rhs": [_vp, _vp, _vpp, ctypes.c_int32, _vp],
    "tt_prox_exact": [_vp, _vp, _vpp, ctypes.c_int32, _vp],
    "tt_als_sweep_exact": [_vp, _vp, _vpp, ctypes.POINTER(ctypes.c_double)],
    "tt_plan_sketch_sources": [_vp, ctypes.POINTER(ctypes.c_int32)],
    "tt_sketch_interface": [_vp, _vpp, ctypes.c_int32, _vp],
    "tt_prox_solve": [_vp, ctypes.c_int32, _vp, _vp, _vp, _vp],
    "tt_left_orth_absorb": [_vp, _vpp, ctypes.c_int32],
    "tt_right_orthogonalize": [_vp, _vpp],
    "tt_residual": [_vp, _vp, _vpp, ctypes.POINTER(ctypes.c_double)],
    "tt_core_change": [_vp, _vpp, _vpp, ctypes.POINTER(ctypes.c_double)],
    "tt_als_sweep": [_vp, _vp, _vpp, ctypes.POINTER(ctypes.c_double)],
    "tt_plan_sync_status": [_vp],
    "tt_plan_profile": [_vp, ctypes.c_int32],
    "tt_plan_profile_read": [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)],
    "tt_plan_sketch_path": [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)],
    "tt_plan_set_overlap": [_vp, ctypes.c_int32],
    "tt_plan_set_sketch": [_vp, ctypes.c_int64, ctypes.c_double],
    "tt_plan_get_sketch": [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)],
    "tt_jpolicy_forward": [_vp, _vp, ctypes.c_int32, _vp, _vp],
    "tt_jpolicy_loss_grad": [_vp, _vp, _vp, ctypes.c_int32, _vp, _vp, _vp],
    "tt_jpolicy_adam": [_vp, _vp, _vp, _vp, ctypes.c_int64, ctypes.c_int64, ctypes.c_float, ctypes.c_float,
                        ctypes.c_float, ctypes.c_float, _vp],
    "tt_jpolicy_features": [_vp, ctypes.c_int64, ctypes.c_double, ctypes.POINTER(ctypes.c_float)],
    "tt_jpolicy_choose": [_vp, _vp, ctypes.c_int64, ctypes.c_double, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64),
                          ctypes.POINTER(ctypes.c_double)],
    "tt_sketch_size_bound": [ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                             ctypes.POINTER(ctypes.c_double)],
    "tt_plan_fallback_J": [_vp, ctypes.c_double, ctypes.c_double, ctypes.POINTER(ctypes.c_int64)],
    "tt_batch_plan": [ctypes.c_int32, _vp, _vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(_vp)],
    "tt_batch_bind_workspace": [_vp, _vp, ctypes.c_size_t],
    "tt_batch_destroy": [_vp],
    "tt_batch_get_plan": [_vp, ctypes.c_int32, ctypes.POINTER(_vp)],
    "tt_batch_set_graph": [_vp, ctypes.c_int32],
    "tt_batch_sketch_tensor": [_vp, _vpp, ctypes.c_int32, _vpp],
    "tt_batch_sweep": [_vp, _vpp, _vp, ctypes.POINTER(ctypes.c_double)],
    "tt_batch_autotune": [_vp, _vpp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)],
    "tt_batch_get_tuning": [_vp, ctypes.POINTER(ctypes.c_int64)],
    "tt_batch_set_tuning": [_vp, ctypes.POINTER(ctypes.c_int64)],
    "tt_batch_sketch_path": [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)],
    "tt_residual_noalloc": [ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                            ctypes.c_int32, ctypes.c_int32, _vp, _vpp, _vp, ctypes.POINTER(ctypes.c_double)],
    "tt_als_run": [_vp, _vp, _vpp, _vp, ctypes.c_int32, ctypes.c_double, ctypes.c_int64, ctypes.POINTER(ctypes.c_double),
                   ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double), ctypes.c_void_p],
}
JPOLICY_FEATURES = 8
JPOLICY_HIDDEN = 64
JPOLICY_OUTPUTS = 2
JPOLICY_PARAMS = 9026
JPOLICY_EXACT_J = 24576        # predictions at or above select the unsketched update
JPOLICY_EXACT_LABEL = 65536    # label of that choice
BATCH_TUNE_FIELDS = 4


class RunStats(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int32), ("reached", ctypes.c_int32), ("fallbacks", ctypes.c_int32),
                ("residual", ctypes.c_double)]


SKETCH_PATHS = {0: "k_sketch_mode0", 1: "k_sketch_modek", 2: "k_sketch_gs"}
BSKETCH_PATHS = {0: "k_bsketch_0", 1: "k_bsketch_k", 2: "k_bsketch_slab", 3: "k_bsketch_ks"}
PROF_CLASSES = ["sketch_k0", "sketch_k", "sketch_aux", "interface", "gram", "solve", "qr", "residual", "tables",
                "exact"]
STRING_FUNCS = ["tt_last_error", "tt_version"]

_lib = None


def load():
    """Load the in-tree HIP library; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libttsketch.so not found at %s: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'`" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    for name, args in SIGNATURES.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    for name in STRING_FUNCS:
        f = getattr(lib, name)
        f.argtypes = []
        f.restype = ctypes.c_char_p
    _lib = lib
    return lib


class TTError(RuntimeError):
    def __init__(self, status, func, msg):
        super().__init__("%s returned %s: %s" % (func, STATUS_NAMES.get(status, status), msg))
        self.status = status


def check(status, func):
    if status != TT_OK:
        raise TTError(status, func, load().tt_last_error().decode())


def ptr_array(ptrs):
    arr = (ctypes.c_void_p * len(ptrs))(*ptrs)
    return ctypes.cast(arr, _vpp), arr
