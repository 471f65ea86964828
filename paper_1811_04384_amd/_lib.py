"""ctypes declarations of the C ABI in include/ising.h (argument marshalling only)."""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libising.so")

c_i32, c_i64, c_u32, c_u64, c_dbl, c_sz = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64,
                                          ctypes.c_double, ctypes.c_size_t)
c_vp, c_int, c_char_p = ctypes.c_void_p, ctypes.c_int, ctypes.c_char_p
P = ctypes.POINTER

ISING_OK, ISING_EINVAL, ISING_ENOMEM, ISING_EHIP, ISING_EBUSY, ISING_EAGAIN = 0, -1, -2, -3, -4, -5
ISING_COLD, ISING_HOT = 0, 1


class BatchPlan(ctypes.Structure):
    _fields_ = [("resident_max_L", c_i32), ("resident_block", c_i32), ("words_per_thread", c_i32),
                ("tiled_block", c_i32), ("sweeps_per_graph", c_i32), ("tile_max_L", c_i32), ("tile_sweeps", c_i32),
                ("tile_cols", c_i32), ("tile_block", c_i32), ("tile_exchange", c_i32),
                ("draw_sweeps", c_i32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class Result(ctypes.Structure):
    _fields_ = [("req_id", c_u64), ("L", c_i32), ("status", c_i32), ("T", c_dbl), ("sweeps", c_i64),
                ("E", c_i64), ("M", c_i64), ("t_submit_s", c_dbl), ("t_admit_s", c_dbl), ("t_done_s", c_dbl)]


class Moments(ctypes.Structure):
    _fields_ = [("n_samples", c_i64), ("sum_E", c_i64), ("sum_E2", c_u64 * 2), ("sum_absM", c_i64),
                ("sum_M2", c_u64 * 2), ("sum_M4", c_u64 * 3)]

    def as_dict(self):
        def wide(limbs):
            return sum(int(v) << (64 * j) for j, v in enumerate(limbs))
        return {"n_samples": int(self.n_samples), "sum_E": int(self.sum_E), "sum_E2": wide(self.sum_E2),
                "sum_absM": int(self.sum_absM), "sum_M2": wide(self.sum_M2), "sum_M4": wide(self.sum_M4)}


class Thermo(ctypes.Structure):
    _fields_ = [("e", c_dbl), ("c", c_dbl), ("abs_m", c_dbl), ("chi", c_dbl), ("binder", c_dbl)]

    def as_dict(self):
        return {k: float(getattr(self, k)) for k, _ in self._fields_}


# name -> (restype, argtypes); every entry point declared in include/ising.h
SIGNATURES = {
    "ising_word_rows": (c_i32, [c_i32]),
    "ising_required_bytes": (c_sz, [c_i32]),
    "ising_thresholds": (c_int, [c_dbl, P(c_u32), P(c_u32)]),
    "ising_version": (c_char_p, []),
    "ising_last_error": (c_char_p, []),
    "ising_create": (c_int, [c_i32, c_u64, c_i32, c_vp, P(c_vp)]),
    "ising_create_in": (c_int, [c_i32, c_u64, c_i32, c_vp, c_sz, c_vp, P(c_vp)]),
    "ising_reset": (c_int, [c_vp, c_u64, c_i32]),
    "ising_destroy": (c_int, [c_vp]),
    "ising_sweep": (c_int, [c_vp, c_dbl, c_i64]),
    "ising_sweep_measure": (c_int, [c_vp, c_dbl, c_i64, c_i32, c_vp, c_vp]),
    "ising_sweep_moments": (c_int, [c_vp, c_dbl, c_i64, c_i32, c_vp]),
    "ising_scan": (c_int, [c_vp, c_i32, P(c_dbl), c_i64, c_i64, c_i32, P(Moments)]),
    "ising_thermodynamics": (c_int, [P(Moments), c_i32, c_dbl, P(Thermo)]),
    "ising_random_iterations": (c_int, [c_vp, c_dbl, c_i32, c_i64, c_i32, c_vp, c_vp, c_vp]),
    "ising_observables": (c_int, [c_vp, P(c_i64), P(c_i64)]),
    "ising_get_spins": (c_int, [c_vp, c_vp]),
    "ising_get_spins_region": (c_int, [c_vp, c_i32, c_i32, c_i32, c_i32, c_vp]),
    "ising_set_spins": (c_int, [c_vp, c_vp]),
    "ising_get_sweep_count": (c_int, [c_vp, P(c_u64)]),
    "ising_set_sweep_count": (c_int, [c_vp, c_u64]),
    "ising_words": (c_int, [c_vp, P(c_vp), P(c_sz)]),
    "ising_set_tiling": (c_int, [c_vp, c_i32, c_i32, c_i32]),
    "ising_get_tiling": (c_int, [c_vp, P(c_i32), P(c_i32), P(c_i32)]),
    "ising_set_resident_tiles": (c_int, [c_vp, c_i32, c_i32, c_i32]),
    "ising_get_resident_tiles": (c_int, [c_vp, P(c_i32), P(c_i32), P(c_i32)]),
    "ising_set_resident_wait": (c_int, [c_vp, ctypes.c_uint64]),
    "ising_sweep_measure_static": (c_int, [c_vp, c_sz, c_i32, c_u64, c_u64, c_dbl, c_i64, c_i32, c_vp, c_vp, c_vp]),
    "ising_set_plan": (c_int, [c_vp, c_i32, c_i32]),
    "ising_get_plan": (c_int, [c_vp, P(c_i32), P(c_i32)]),
    "ising_autotune": (c_int, [c_vp, c_dbl, P(c_dbl)]),
    "ising_synchronize": (c_int, [c_vp]),
    "ising_batch_create": (c_int, [c_i32, P(c_i32), P(c_u64), P(c_i32), c_vp, P(c_vp)]),
    "ising_batch_destroy": (c_int, [c_vp]),
    "ising_batch_sweep": (c_int, [c_vp, P(c_dbl), c_i64, c_i32, c_vp, c_vp]),
    "ising_batch_results": (c_int, [c_vp, P(c_i64), P(c_i64), P(c_i64), P(c_i64), P(c_i64)]),
    "ising_batch_reset_sums": (c_int, [c_vp]),
    "ising_batch_moments": (c_int, [c_vp, P(Moments)]),
    "ising_batch_scan": (c_int, [c_vp, c_i32, P(c_dbl), c_i64, c_i64, c_i32, P(Moments)]),
    "ising_batch_get_spins": (c_int, [c_vp, c_i32, c_vp]),
    "ising_batch_get_spins_region": (c_int, [c_vp, c_i32, c_i32, c_i32, c_i32, c_i32, c_vp]),
    "ising_batch_get_sweep_count": (c_int, [c_vp, c_i32, P(c_u64)]),
    "ising_batch_check_plan": (c_int, [P(BatchPlan)]),
    "ising_batch_set_plan": (c_int, [c_vp, P(BatchPlan)]),
    "ising_batch_get_plan": (c_int, [c_vp, P(BatchPlan)]),
    "ising_batch_autotune": (c_int, [c_vp, P(c_dbl), c_char_p, P(BatchPlan)]),
    "ising_replicas_create": (c_int, [c_i32, c_u64, c_i32, c_vp, P(c_vp)]),
    "ising_replicas_destroy": (c_int, [c_vp]),
    "ising_replicas_sweep": (c_int, [c_vp, P(c_dbl), c_i64]),
    "ising_replicas_sweep_measure": (c_int, [c_vp, P(c_dbl), c_i64, c_i32, c_vp, c_vp]),
    "ising_replicas_sweep_moments": (c_int, [c_vp, P(c_dbl), c_i64, c_i32, c_vp]),
    "ising_replicas_observables": (c_int, [c_vp, P(c_i64), P(c_i64)]),
    "ising_replicas_get_spins": (c_int, [c_vp, c_i32, c_vp]),
    "ising_replicas_get_sweep_count": (c_int, [c_vp, P(c_u64)]),
    "ising_replicas_set_plan": (c_int, [c_vp, c_i32]),
    "ising_server_create": (c_int, [c_sz, c_i32, c_i32, c_vp, P(c_vp)]),
    "ising_server_submit": (c_int, [c_vp, c_u64, c_i32, c_dbl, c_i64, c_u64, c_i32]),
    "ising_server_step": (c_int, [c_vp, P(c_i32)]),
    "ising_server_poll": (c_int, [c_vp, P(Result), c_i32, P(c_i32)]),
    "ising_server_stats": (c_int, [c_vp, P(c_i32), P(c_i32), P(c_i32), P(c_sz)]),
    "ising_server_destroy": (c_int, [c_vp]),
}

_lib = None


def load():
    """Load libising.so.  There is no fallback: a missing or stale library is
    an error (build it with ``python -m paper_1811_04384_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1811_04384_amd.build` first")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)  # AttributeError here means the library lacks an entry point
        fn.restype = res
        fn.argtypes = args
    from .build import source_hash

    version = lib.ising_version().decode()
    if not version.endswith(" src " + source_hash()):
        raise ImportError(f"{LIB_PATH} ({version}) was built from other sources than the ones beside it; "
                          "rebuild with `python -m paper_1811_04384_amd.build`")
    _lib = lib
    return lib
