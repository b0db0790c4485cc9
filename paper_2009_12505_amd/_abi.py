"""ctypes mirror of include/hfx.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhfx.so")

HFX_OK, HFX_ERR_ARG, HFX_ERR_SHAPE, HFX_ERR_SYMMETRY, HFX_ERR_OOM, HFX_ERR_HIP, HFX_ERR_STATE, \
    HFX_ERR_UNSUPPORTED = range(8)
STATUS_NAMES = ["HFX_OK", "HFX_ERR_ARG", "HFX_ERR_SHAPE", "HFX_ERR_SYMMETRY", "HFX_ERR_OOM", "HFX_ERR_HIP",
                "HFX_ERR_STATE", "HFX_ERR_UNSUPPORTED"]

PREC_FP64, PREC_FP32, PREC_TIERED, PREC_BF16X3 = 0, 1, 2, 3
SCREEN_PRE, SCREEN_CS_ERI, SCREEN_CS1, SCREEN_CS2, SCREEN_CS3 = 1, 2, 4, 8, 16
SCREEN_ALL = 31
SCHED_PLAN, SCHED_LPT, SCHED_MLP, SCHED_EXACT, SCHED_NORM, SCHED_KMEANS = 0, 1, 2, 3, 4, 5

EXPORTED = ["hfx_plan_create", "hfx_sigma_layout", "hfx_build", "hfx_energy", "hfx_item_profile",
            "hfx_plan_destroy", "hfx_last_error", "hfx_abi_version", "hfx_mlp_n_params", "hfx_mlp_predict",
            "hfx_mlp_loss_grad", "hfx_mlp_train", "hfx_item_features", "hfx_sigma_to_k",
            "hfx_density_from_k", "hfx_mlp_train_static", "hfx_tune_key", "hfx_mfma_peak"]
ITEM_UNITS = 5
ITEM_FEATURES = 10
ITEM_TARGETS = 2
ABI_VERSION = 3


class Species(ctypes.Structure):
    _fields_ = [("n_ao", ctypes.c_int32), ("n_abf", ctypes.c_int32)]


class Cell(ctypes.Structure):
    _fields_ = [("n_atoms", ctypes.c_int32), ("lattice", ctypes.c_double * 9), ("pos", ctypes.c_void_p),
                ("species", ctypes.c_void_p), ("n_species", ctypes.c_int32), ("sp", ctypes.POINTER(Species))]


class Blocks(ctypes.Structure):
    _fields_ = [("n_blocks", ctypes.c_int64), ("row", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("R", ctypes.c_void_p), ("off", ctypes.c_void_p), ("data", ctypes.c_void_p),
                ("on_device", ctypes.c_int32)]


class Thresholds(ctypes.Structure):
    _fields_ = [("eps_C", ctypes.c_double), ("eps_V", ctypes.c_double), ("eps_D", ctypes.c_double),
                ("eps_cs_eri", ctypes.c_double), ("eps_cs_mat", ctypes.c_double)]


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("stages", ctypes.c_uint32), ("tier_tau", ctypes.c_double),
                ("tier_tau_bf", ctypes.c_double), ("scheduler", ctypes.c_int32), ("mlp_weights", ctypes.c_char_p),
                ("stream", ctypes.c_void_p), ("home_subset", ctypes.c_void_p), ("n_home_subset", ctypes.c_int32),
                ("max_device_bytes", ctypes.c_uint64), ("n_slots", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("tuning_db", ctypes.c_char_p), ("tile_r", ctypes.c_int32)]


class BuildStats(ctypes.Structure):
    _fields_ = [("candidates", ctypes.c_int64), ("kept_cs_eri", ctypes.c_int64),
                ("kept", (ctypes.c_int64 * 4) * 3), ("items", ctypes.c_int64), ("g_alive", ctypes.c_int64),
                ("flops_contract", ctypes.c_double), ("flops_paper", ctypes.c_double),
                ("flops_tier", ctypes.c_double * 3), ("mfma_flops", ctypes.c_double * 3),
                ("ms_total", ctypes.c_double), ("ms_main", ctypes.c_double),
                ("phase_share", ctypes.c_double * 6), ("mfma_flops_fp32", ctypes.c_double),
                ("tile_r", ctypes.c_int32), ("pad", ctypes.c_int32), ("tier_tau", ctypes.c_double),
                ("tier_tau_bf", ctypes.c_double), ("mfma_flops_bf16", ctypes.c_double)]

    def as_dict(self) -> dict:
        d = {"candidates": self.candidates, "kept_cs_eri": self.kept_cs_eri, "items": self.items,
             "g_alive": self.g_alive, "flops_contract": self.flops_contract, "flops_paper": self.flops_paper,
             "flops_tier": list(self.flops_tier), "mfma_flops": list(self.mfma_flops),
             "ms_total": self.ms_total, "ms_main": self.ms_main, "mfma_flops_fp32": self.mfma_flops_fp32,
             "tile_r": self.tile_r, "tier_tau": self.tier_tau, "tier_tau_bf": self.tier_tau_bf,
             "mfma_flops_bf16": self.mfma_flops_bf16,
             "phase_share": dict(zip(["screen", "gside", "masks", "gemm_r", "gemm_l", "setup"],
                                     [round(x, 4) for x in self.phase_share]))}
        for s in range(3):
            for t in range(4):
                d[f"kept_s{s + 1}_t{t + 1}"] = self.kept[s][t]
        return d


_lib = None


class HfxError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES[status] if 0 <= status < 8 else status}: {msg}")
        self.status = status


def lib():
    """Load libhfx.so; raises if the HIP library has not been built."""
    global _lib
    if _lib is None:
        # torch first: it maps its own HIP runtime (same soname), which the library must then share;
        # loaded the other way round, the process would hold two runtimes whose device pointers and
        # streams are not interchangeable
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2009_12505_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.hfx_plan_create.restype = ctypes.c_int
        L.hfx_plan_create.argtypes = [ctypes.c_int32, P, P, P, P, P, P, ctypes.POINTER(P)]
        L.hfx_sigma_layout.restype = ctypes.c_int
        L.hfx_sigma_layout.argtypes = [P, ctypes.c_int32, ctypes.POINTER(Blocks), ctypes.POINTER(ctypes.c_int64)]
        L.hfx_build.restype = ctypes.c_int
        L.hfx_build.argtypes = [P, P, P, P]
        L.hfx_energy.restype = ctypes.c_int
        L.hfx_energy.argtypes = [P, P, P, P]
        L.hfx_item_profile.restype = ctypes.c_int
        L.hfx_item_profile.argtypes = [P, ctypes.POINTER(ctypes.c_int64), P, P, P]
        L.hfx_plan_destroy.restype = None
        L.hfx_plan_destroy.argtypes = [P]
        L.hfx_last_error.restype = ctypes.c_char_p
        L.hfx_last_error.argtypes = []
        L.hfx_abi_version.restype = ctypes.c_int32
        L.hfx_abi_version.argtypes = []
        L.hfx_mlp_n_params.restype = ctypes.c_int64
        L.hfx_mlp_n_params.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        L.hfx_mlp_predict.restype = ctypes.c_int
        L.hfx_mlp_predict.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, P, ctypes.c_int64, P, P]
        L.hfx_mlp_loss_grad.restype = ctypes.c_int
        L.hfx_mlp_loss_grad.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, P, P, ctypes.c_int64, P, P,
                                        P]
        L.hfx_mlp_train.restype = ctypes.c_int
        L.hfx_mlp_train.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, P, P, ctypes.c_int64, ctypes.c_int32,
                                    ctypes.c_float, P, P]
        L.hfx_mlp_train_static.restype = ctypes.c_int
        L.hfx_mlp_train_static.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, P, P, ctypes.c_int64,
                                           ctypes.c_int32, ctypes.c_float, P, P]
        L.hfx_tune_key.restype = ctypes.c_int
        L.hfx_tune_key.argtypes = [P, ctypes.c_char_p, ctypes.c_int32]
        L.hfx_item_features.restype = ctypes.c_int
        L.hfx_item_features.argtypes = [P, P, P, P]
        L.hfx_sigma_to_k.restype = ctypes.c_int
        L.hfx_sigma_to_k.argtypes = [P, ctypes.c_int32, P, ctypes.c_int32, P, P]
        L.hfx_mfma_peak.restype = ctypes.c_int
        L.hfx_mfma_peak.argtypes = [ctypes.c_int32, P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.hfx_density_from_k.restype = ctypes.c_int
        L.hfx_density_from_k.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P, ctypes.c_int32, P, P, P]
        if L.hfx_abi_version() != ABI_VERSION:
            raise ImportError(f"{LIB_PATH} has ABI version {L.hfx_abi_version()}, this binding expects "
                              f"{ABI_VERSION}: rebuild it with `python -m paper_2009_12505_amd.build`")
        _lib = L
    return _lib


def check(status: int):
    if status != HFX_OK:
        raise HfxError(status, lib().hfx_last_error().decode())
