"""ctypes binding of libmbc (include/mbc.h, mbc_blocks.h, mbc_egraph.h, mbc_tree.h): argument marshalling only.

Every step of the contraction runs in the library; this module only converts
Python/torch arguments to pointers and sizes and raises on a non-zero status.
Loading fails loudly when the library has not been built.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libmbc.so")

MBC_OK = 0
MBC_ERR_UNSUPPORTED = 2
OPS = {"proton": 0, "neutron": 1, "DI": 2, "DII": 3, "HE3_I": 4, "HE3_II": 5}
SIGNS = {"exact": 0, "r2": 1}
F64, F32C = 0, 1
C128, C64 = 0, 1


class MbcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libmbc status {status}: {msg}")
        self.status = status


class OpDesc(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("snk_spin", ctypes.c_int32), ("src_spin", ctypes.c_int32),
                ("sign_mode", ctypes.c_int32), ("symmetrise", ctypes.c_int32)]


class PlanStats(ctypes.Structure):
    _fields_ = [("nnz", ctypes.c_int64), ("n_corr", ctypes.c_int32), ("n_u", ctypes.c_int32),
                ("n_d", ctypes.c_int32), ("precision", ctypes.c_int32), ("n_tiles", ctypes.c_int32),
                ("threads", ctypes.c_int32), ("lds_bytes", ctypes.c_int64),
                ("alg_flops_per_site", ctypes.c_double), ("exec_flops_per_site", ctypes.c_double),
                ("in_bytes_per_site", ctypes.c_double), ("b_n_tiles", ctypes.c_int32),
                ("b_lds_bytes_ds", ctypes.c_int64), ("b_lds_bytes_dw", ctypes.c_int64),
                ("ds_alg_flops_per_site", ctypes.c_double), ("dw_alg_flops_per_site", ctypes.c_double),
                ("w_n_tiles", ctypes.c_int32), ("rank1", ctypes.c_int32), ("f_n_tiles", ctypes.c_int32),
                ("f_lds_bytes_ds", ctypes.c_int64), ("fwd_factored", ctypes.c_int32), ("ds_factored", ctypes.c_int32),
                ("f_lds_bytes_fwd", ctypes.c_int64), ("fact_alg_flops_per_site", ctypes.c_double),
                ("fact_ds_alg_flops_per_site", ctypes.c_double)]


class BlockCorrDesc(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("snk_spin", ctypes.c_int32), ("src_spin", ctypes.c_int32),
                ("sign_mode", ctypes.c_int32), ("mom", (ctypes.c_int32 * 3) * 3), ("src_pt", ctypes.c_int32 * 3)]


class BlockPlanStats(ctypes.Structure):
    _fields_ = [("n_types", ctypes.c_int32), ("n_slots", ctypes.c_int32), ("n_corr", ctypes.c_int32),
                ("n_points", ctypes.c_int32), ("n_terms", ctypes.c_int64), ("n_gmats", ctypes.c_int32),
                ("block_flops_per_site", ctypes.c_double),
                ("contract_flops_per_t", ctypes.c_double), ("tree_vertices", ctypes.c_int64),
                ("tree_flops_per_t", ctypes.c_double)]


class TensorDecl(ctypes.Structure):
    _fields_ = [("rank", ctypes.c_int32), ("ext", ctypes.c_int32 * 8), ("n_sym", ctypes.c_int32),
                ("perm", (ctypes.c_int32 * 8) * 4), ("sign", ctypes.c_int32 * 4)]


class TensorFactor(ctypes.Structure):
    _fields_ = [("tensor", ctypes.c_int32), ("label", ctypes.c_int32 * 8)]


class EGraphStats(ctypes.Structure):
    _fields_ = [("n_tensors", ctypes.c_int32), ("n_terms", ctypes.c_int32), ("n_classes", ctypes.c_int32),
                ("n_nodes", ctypes.c_int32), ("saturated", ctypes.c_int32), ("n_roots", ctypes.c_int32),
                ("n_steps", ctypes.c_int32), ("n_open", ctypes.c_int32), ("out_ext", ctypes.c_int32 * 64),
                ("out_elems", ctypes.c_int64), ("ws_elems", ctypes.c_int64),
                ("flops_direct", ctypes.c_double), ("flops_plan", ctypes.c_double)]


EXTRACT = {"reuse": 0, "flops": 1, "shared": 2}
FAMILIES = {0: "p", 1: "n"}
BLOCK_METHODS = {"terms": 0, "tree": 1}

_lib = None

# exported symbols and their signatures: (name, restype, argtypes)
_P, _I32, _I64, _SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
SIGNATURES = [
    ("mbc_last_error", ctypes.c_char_p, []),
    ("mbc_version", ctypes.c_char_p, []),
    ("mbc_build_index_set", _I32, [ctypes.POINTER(OpDesc), _I32, ctypes.POINTER(_P)]),
    ("mbc_index_set_dims", _I32, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                                  ctypes.POINTER(_I64), ctypes.POINTER(_I32)]),
    ("mbc_index_set_export", _I32, [_P] + [_P] * 8),
    ("mbc_index_set_free", None, [_P]),
    ("mbc_plan_create", _I32, [_P, _I32, _P, ctypes.POINTER(_P)]),
    ("mbc_plan_get_stats", _I32, [_P, ctypes.POINTER(PlanStats)]),
    ("mbc_plan_workspace_bytes", _I32, [_P, _I32, _I64, _I32, ctypes.POINTER(_SZ)]),
    ("mbc_plan_destroy", None, [_P]),
    ("mbc_contract", _I32, [_P, _P, _P, _I32, _I32, _I64, _P, _P, _P, _SZ, _P]),
    ("mbc_contract_noalloc", _I32, [_P, _P, _P, _I32, _I32, _I64, _P, _P, _P]),
    ("mbc_contract_backward", _I32, [_P, _P, _P, _I32, _I32, _I64, _P, _P, _P, _P, _P, _P, _SZ, _P]),
    ("mbc_debug_eval_host", _I32, [_P, _I32, _P, _P, _I32, _I64, _P, _P, ctypes.POINTER(PlanStats)]),
    ("mbc_debug_backward_host", _I32, [_P, _I32, _P, _P, _I32, _I64, _P, _P, _P, _P, _P]),
    ("mbc_block_set_build", _I32, [ctypes.POINTER(BlockCorrDesc), _I32, ctypes.POINTER(_P)]),
    ("mbc_block_set_dims", _I32, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                                  ctypes.POINTER(_I64), ctypes.POINTER(_I32)]),
    ("mbc_block_set_types", _I32, [_P, _P, _P, _P, _P]),
    ("mbc_block_set_export", _I32, [_P] * 6),
    ("mbc_block_set_factor_tree", _I32, [_P, _I32, ctypes.POINTER(_I64), _P, _P]),
    ("mbc_block_set_free", None, [_P]),
    ("mbc_block_multiplicities", _I32, [ctypes.POINTER(BlockCorrDesc), _I64, ctypes.POINTER(_I64),
                                        ctypes.POINTER(_I64), ctypes.POINTER(_I64), _P, _I32]),
    ("mbc_block_plan_create", _I32, [_P, _P, ctypes.POINTER(_P)]),
    ("mbc_block_plan_get_stats", _I32, [_P, ctypes.POINTER(BlockPlanStats)]),
    ("mbc_block_workspace_bytes", _I32, [_P, _I32, _P, ctypes.POINTER(_SZ)]),
    ("mbc_block_plan_destroy", None, [_P]),
    ("mbc_blocks_compute", _I32, [_P, _P, _P, _I32, _I32, _P, _P, _P, _SZ, _P]),
    ("mbc_block_contract", _I32, [_P, _P, _I32, _I32, _P, _P, _SZ, _P]),
    ("mbc_egraph_build", _I32, [ctypes.POINTER(TensorDecl), _I32, ctypes.POINTER(TensorFactor), _P, _P, _I32,
                                _I64, _I32, ctypes.POINTER(_P)]),
    ("mbc_egraph_build_blocks", _I32, [_P, _I32, _I64, _I32, ctypes.POINTER(_P)]),
    ("mbc_egraph_get_stats", _I32, [_P, ctypes.POINTER(EGraphStats)]),
    ("mbc_egraph_export", _I32, [_P, _P, _I64, ctypes.POINTER(_I64)]),
    ("mbc_egraph_term_coefs", _I32, [_P, _P]),
    ("mbc_egraph_workspace_bytes", _I32, [_P, _I64, ctypes.POINTER(_SZ)]),
    ("mbc_egraph_execute", _I32, [_P, _P, _P, _I64, _P, _P, _SZ, _P]),
    ("mbc_egraph_free", None, [_P]),
    ("mbc_factor_tree_create", _I32, [_P, _P, _I64, _P, _I64, _I32, _P, ctypes.POINTER(_P)]),
    ("mbc_factor_tree_stats", _I32, [_P, ctypes.POINTER(_I32), ctypes.POINTER(ctypes.c_double)]),
    ("mbc_factor_tree_workspace_bytes", _I32, [_P, _I64, ctypes.POINTER(_SZ)]),
    ("mbc_factor_tree_evaluate", _I32, [_P, _P, _I64, _P, _P, _SZ, _P]),
    ("mbc_factor_tree_destroy", None, [_P]),
]


def lib():
    """The loaded library; raises if libmbc.so has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2201_04269_amd.build` (there is no fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status):
    if status != MBC_OK:
        raise MbcError(status, lib().mbc_last_error().decode())
