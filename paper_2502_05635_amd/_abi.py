"""ctypes mirror of include/tdagw.h (structs, constants, signatures)."""

import ctypes as C

TDG_OK = 0
TDG_E_INVAL = -1
TDG_E_HIP = -2
TDG_E_NOMEM = -3
TDG_E_UNSUPPORTED = -4
TDG_E_NUMERIC = -5
TDG_E_SOLVER = -6

TDG_C128 = 0
TDG_C64 = 1
TDG_BF16X2 = 2
TDG_BLOCK_ALL = 0
TDG_BLOCK_EH = 1
TDG_NB_MAX = 8
TDG_TRUNC = {"rel_cut": 0, "fraction": 1, "rank": 2, "r2": 3}
TDG_OP_DENSE = 0
TDG_OP_LOWRANK = 1
TDG_OP_CHANNEL = 2
TDG_KCLASS_STAGE = 0
TDG_KCLASS_PROJECT = 1
TDG_KCLASS_GEMM = 2
TDG_KCLASS_INTRA = 3
TDG_OPT_AUTOTUNE = 0
TDG_OPT_STAGE_VARIANT = 1
TDG_OPT_BATCHED_MIN = 2
TDG_OPT_GEMM_TILE = 3
TDG_OPT_GEMM_VARIANT = 4
TDG_OPT_GRAPHS = 5
TDG_OPT_GEMM_SLICES = 6
TDG_OPT_ADJOINT_STASH = 7
TDG_NOALLOC_SCRATCH_BYTES = 33554432

P = C.c_void_p


class Model(C.Structure):
    _fields_ = [("nk1", C.c_int32), ("nk2", C.c_int32), ("nb", C.c_int32), ("nv", C.c_int32),
                ("shift", C.c_double), ("a_bohr", C.c_double),
                ("eps", P), ("evec", P), ("dip", P), ("vel", P), ("links", P)]


class Coulomb(C.Structure):
    _fields_ = [("r0_bohr", C.c_double), ("block", C.c_int32), ("nquad", C.c_int32)]


class Trunc(C.Structure):
    _fields_ = [("mode", C.c_int32), ("pad", C.c_int32), ("value", C.c_double)]


class LowRank(C.Structure):
    _fields_ = [("n", C.c_int64), ("max_rank", C.c_int64), ("dtype", C.c_int32), ("pad", C.c_int32),
                ("kdiag", P), ("us", P), ("w", P), ("sigma", P),
                ("rank", C.c_int64), ("tail_fro", C.c_double), ("tail_spec", C.c_double)]


class Channels(C.Structure):
    _fields_ = [("nk", C.c_int64), ("npair", C.c_int32), ("dtype", C.c_int32), ("rmax", C.c_int64),
                ("diag", P), ("s", P), ("w", P), ("ranks", P), ("sigma", P)]


class Field(C.Structure):
    _fields_ = [("e0", C.c_double), ("omega", C.c_double), ("tau", C.c_double), ("t0", C.c_double),
                ("ex", C.c_double), ("ey", C.c_double), ("nsteps", C.c_double), ("pad", C.c_double)]


class Operator(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dtype", C.c_int32), ("block", C.c_int32), ("pad", C.c_int32),
                ("n", C.c_int64), ("K", P), ("ld", C.c_int64),
                ("kdiag", P), ("us", P), ("w", P), ("rank", C.c_int64)]


class Obs(C.Structure):
    _fields_ = [("P", P), ("J", P), ("occ", P), ("tr", P), ("herm", P), ("stride", C.c_int64)]


class ObsGrad(C.Structure):
    _fields_ = [("gP", P), ("gJ", P), ("gocc", P), ("stride", C.c_int64)]


class Grads(C.Structure):
    _fields_ = [("dfield", P), ("dE", P), ("drho0", P), ("dus", P), ("dw", P)]


SIGNATURES = {
    "tdg_version": ([], C.c_int),
    "tdg_create": ([C.POINTER(P), C.c_int, P], C.c_int),
    "tdg_destroy": ([P], C.c_int),
    "tdg_set_stream": ([P, P], C.c_int),
    "tdg_last_error": ([P], C.c_char_p),
    "tdg_kernel_dim": ([C.POINTER(Model), C.c_int32, C.POINTER(C.c_int64)], C.c_int),
    "tdg_links_build": ([P, C.POINTER(Model), P], C.c_int),
    "tdg_kernel_build": ([P, C.POINTER(Model), C.POINTER(Coulomb), C.c_int32, P, C.c_int64], C.c_int),
    "tdg_kernel_compress": ([P, P, C.c_int64, C.c_int32, C.POINTER(Trunc), C.POINTER(LowRank)], C.c_int),
    "tdg_kernel_compress_randomized": ([P, P, C.c_int64, C.c_int32, C.POINTER(Trunc), P, C.c_int64, C.c_int32,
                                        C.POINTER(LowRank)], C.c_int),
    "tdg_kernel_compress_channels": ([P, P, C.c_int64, C.c_int32, C.POINTER(Trunc), C.POINTER(Channels)], C.c_int),
    "tdg_propagate": ([P, C.POINTER(Operator), C.POINTER(Model), C.POINTER(Field), C.c_int32, C.c_double, P,
                       C.c_int32, C.POINTER(Obs)], C.c_int),
    "tdg_propagate_noalloc": ([P, C.POINTER(Operator), C.POINTER(Model), C.POINTER(Field), C.c_int32, C.c_double, P,
                               C.c_int32, C.POINTER(Obs)], C.c_int),
    "tdg_propagate_adjoint": ([P, C.POINTER(Operator), C.POINTER(Model), C.POINTER(Field), C.c_int32, C.c_double,
                               P, C.c_int32, C.POINTER(ObsGrad), C.POINTER(Grads)], C.c_int),
    "tdg_observables": ([P, C.POINTER(Model), P, C.c_int32, C.POINTER(Field), P], C.c_int),
    "tdg_check_numeric": ([P, C.POINTER(Obs), C.c_int32, C.POINTER(Field), C.c_double, C.c_double], C.c_int),
    "tdg_set_option": ([P, C.c_int32, C.c_int64], C.c_int),
    "tdg_last_variant": ([P], C.c_char_p),
    "tdg_profile_enable": ([P, C.c_int32], C.c_int),
    "tdg_profile_read": ([P, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64)], C.c_int),
}
