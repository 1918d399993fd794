"""ctypes declarations of the C ABI in include/hssx.h.  Loading fails loudly
when libhssx.so has not been built; there is no fallback implementation."""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhssx.so")

HSSX_OK, HSSX_ENOCONV = 0, 1
HSSX_EINVAL, HSSX_ENOMEM, HSSX_ESINGULAR, HSSX_ERANKCAP, HSSX_EHIP = -1, -2, -3, -4, -5
HSSX_C128, HSSX_C64 = 0, 1

STATUS_NAMES = {0: "HSSX_OK", 1: "HSSX_ENOCONV", -1: "HSSX_EINVAL", -2: "HSSX_ENOMEM",
                -3: "HSSX_ESINGULAR", -4: "HSSX_ERANKCAP", -5: "HSSX_EHIP"}


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


class ProblemDesc(C.Structure):
    _fields_ = [("N", C.c_int), ("omega", C.c_double)]


class IpdgDesc(C.Structure):
    _fields_ = [("N", C.c_int), ("p", C.c_int), ("bc", C.c_int), ("omega", C.c_double)]


BC_ABSORBING, BC_DIRICHLET = 0, 1


class FactorOpts(C.Structure):
    _fields_ = [("beta", C.c_int), ("h_sw", C.c_int), ("k0", C.c_int), ("r", C.c_int),
                ("max_rounds", C.c_int), ("dtype", C.c_int), ("seed", C.c_uint32),
                ("id_rel_tol", C.c_double), ("apply_graph", C.c_int), ("autotune", C.c_int),
                ("sample_bf16", C.c_int), ("switch_size", C.c_int), ("strict_tol", C.c_int),
                ("wide_inverse", C.c_int)]


class GmresOpts(C.Structure):
    _fields_ = [("m", C.c_int), ("tol", C.c_double), ("maxit", C.c_int), ("flexible", C.c_int)]


class GmresStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("converged", C.c_int), ("prec_res", C.c_double),
                ("true_res", C.c_double)]


class FactorStats(C.Structure):
    _fields_ = [("n", C.c_int), ("nodes", C.c_int), ("depth", C.c_int),
                ("n_hss_nodes", C.c_int), ("n_compressed", C.c_int), ("k_max", C.c_int),
                ("max_rounds_used", C.c_int), ("max_estimate", C.c_double),
                ("factor_bytes", C.c_double), ("factor_flops", C.c_double),
                ("ms_symbolic", C.c_double), ("ms_numeric", C.c_double),
                ("ms_setup", C.c_double), ("rounds_total", C.c_int),
                ("n_above_tol", C.c_int), ("exact_factor_bytes", C.c_double),
                ("exact_factor_flops", C.c_double)]


_vp = C.c_void_p
_i = C.c_int
_l = C.c_long
_d = C.c_double
_ip = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_dp = C.POINTER(C.c_double)

SIGNATURES = {
    "hssx_assemble": (_i, [_i, C.POINTER(ProblemDesc), _vp, _vp, C.POINTER(_vp)]),
    "hssx_assemble_elastic": (_i, [_i, C.POINTER(ProblemDesc), _vp, _vp, _vp, _vp,
                                   C.POINTER(_vp)]),
    "hssx_op_batch": (_i, [_i, C.POINTER(_vp), _vp, C.POINTER(_vp)]),
    "hssx_op_info": (_i, [_vp, C.POINTER(_i), C.POINTER(_i), _ip]),
    "hssx_load": (_i, [_vp, _i, _vp, _l, _vp, _l, _vp]),
    "hssx_matvec": (_i, [_vp, _i, _i, _vp, _l, _vp, _l, _vp]),
    "hssx_get_csr": (_i, [_vp, _ip, _ip, _dp, C.POINTER(_l), _vp]),
    "hssx_factor": (_i, [_vp, _d, _i, C.POINTER(FactorOpts), _vp, C.POINTER(_vp)]),
    "hssx_apply": (_i, [_vp, _i, _i, _vp, _l, _vp, _l, _vp]),
    "hssx_apply_noalloc": (_i, [_vp, _i, _i, _vp, _l, _vp, _l, _vp]),
    "hssx_gmres_solve": (_i, [_vp, _vp, _i, _i, _vp, _l, _vp, _l, C.POINTER(GmresOpts),
                              C.POINTER(GmresStats), _vp]),
    "hssx_dAds_contract": (_i, [_vp, _i, _vp, _vp, _vp, _vp]),
    "hssx_dAds_contract_adjoint": (_i, [_vp, _i, _vp, _vp, _vp, _vp]),
    "hssx_analyze": (_i, [_i, _i, _i, _i, C.POINTER(_vp)]),
    "hssx_analyze_dg": (_i, [_i, _i, _i, C.POINTER(_vp)]),
    "hssx_analyze_ipdg": (_i, [_i, _i, _i, _i, C.POINTER(_vp)]),
    "hssx_refactor": (_i, [_vp, _vp, _vp]),
    "hssx_assemble_dg": (_i, [_i, C.POINTER(ProblemDesc), _vp, _vp, C.POINTER(_vp)]),
    "hssx_assemble_ipdg": (_i, [_i, C.POINTER(IpdgDesc), _vp, _vp, C.POINTER(_vp)]),
    "hssx_get_perm": (_i, [_vp, _ip, _l]),
    "hssx_get_tree": (_i, [_vp, _i64p, _ip, _ip, _ip, _ip, _ip, _ip, _ip]),
    "hssx_get_factor_stats": (_i, [_vp, C.POINTER(FactorStats)]),
    "hssx_get_schur": (_i, [_vp, _i, _dp, _l]),
    "hssx_hss_eval": (_i, [_i, _i, _i, _i, _ip, _ip, _dp, _i, _i, _vp, _vp, _l, _ip, _dp, _vp]),
    "hssx_create": (_i, [_i, _vp, C.POINTER(_vp)]),
    "hssx_bind": (_i, [_vp]),
    "hssx_ctx_stats": (_i, [_vp, C.POINTER(_l), C.POINTER(_l), C.POINTER(_l)]),
    "hssx_destroy": (None, [_vp]),
    "hssx_prof_enable": (_i, [_i]),
    "hssx_prof_query": (_i, [C.c_char_p, _dp, C.POINTER(_l), _dp]),
    "hssx_fact_destroy": (None, [_vp]),
    "hssx_op_destroy": (None, [_vp]),
    "hssx_last_error": (C.c_char_p, []),
}

_LIB = None


def lib():
    """The loaded library with argument/return types declared."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2105_07791_amd.build` "
                "(there is no non-HIP implementation of this package)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


class HssxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(code):
    if code < 0:
        raise HssxError(code, lib().hssx_last_error().decode())
    return code
