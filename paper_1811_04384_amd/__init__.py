"""MI355X (gfx950) multi-spin-coded checkerboard Metropolis for the 2D Ising model.

Thin Python binding of the C ABI in ``include/ising.h`` (``libising.so``, built
in-tree by ``python -m paper_1811_04384_amd.build``).  Every step of the
method runs in the library's HIP kernels; this module only marshals
arguments.  PyTorch supplies device memory and the stream.  There is no CPU
fallback: if the library is missing, importing the functions raises.

Functions carry the C names (``ising_create``, ``ising_sweep``,
``ising_observables``, ...); the classes ``Lattice``, ``Batch`` and ``Server``
wrap handles for convenience.
"""
import ctypes

import numpy as np

from . import _lib
from ._lib import (ISING_COLD, ISING_EAGAIN, ISING_EBUSY, ISING_EHIP, ISING_EINVAL, ISING_ENOMEM, ISING_HOT, ISING_OK,
                   BatchPlan, Moments, Result, Thermo)

__all__ = [
    "IsingError", "Lattice", "Batch", "Replicas", "Server", "BatchPlan", "Result", "Moments", "Thermo", "load",
    "moments_of", "REPLICAS",
    "ISING_OK", "ISING_EINVAL", "ISING_ENOMEM", "ISING_EHIP", "ISING_EBUSY", "ISING_EAGAIN", "ISING_COLD", "ISING_HOT",
] + sorted(_lib.SIGNATURES)


class IsingError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def load():
    """The loaded ctypes library (raises ImportError if it is not built)."""
    return _lib.load()


def _check(rc):
    if rc != ISING_OK:
        raise IsingError(rc, _lib.load().ising_last_error().decode())
    return rc


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


class _Ordering:
    """Orders torch's current stream and a handle's own stream around a call
    that enqueues library work: before it, the library's stream waits for
    what torch has enqueued (e.g. the zeroing of an accumulator); after it,
    torch's current stream waits for the library's work, and the output
    tensors are marked as used on the library's stream, so that neither a
    read through torch nor the caching allocator's reuse can overtake the
    kernels that write them.  Nothing to do when the handle uses torch's
    current stream."""

    def __init__(self, stream):
        self.stream = stream

    def _lib(self):
        import torch

        if self.stream is None:
            return None
        if isinstance(self.stream, torch.cuda.Stream):
            s = self.stream
        elif hasattr(self.stream, "cuda_stream"):
            s = torch.cuda.ExternalStream(self.stream.cuda_stream)
        else:
            s = torch.cuda.ExternalStream(int(self.stream))
        return None if s.cuda_stream == torch.cuda.current_stream().cuda_stream else s

    def before(self):
        import torch

        s = self._lib()
        if s is not None:
            s.wait_stream(torch.cuda.current_stream())

    def after(self, *tensors):
        import torch

        s = self._lib()
        if s is None:
            return
        for t in tensors:
            if t is not None:
                t.record_stream(s)
        torch.cuda.current_stream().wait_stream(s)


def _ptr(x):
    """Device or host address of a torch tensor / numpy array / int / None."""
    if x is None:
        return None
    if isinstance(x, int):
        return ctypes.c_void_p(x)
    if hasattr(x, "data_ptr"):
        return ctypes.c_void_p(x.data_ptr())
    if isinstance(x, np.ndarray):
        return ctypes.c_void_p(x.ctypes.data)
    raise TypeError(f"cannot pass {type(x)} as a pointer")


def _arr(a, ctype):
    a = np.ascontiguousarray(a, dtype=np.dtype(ctype))
    return a, a.ctypes.data_as(ctypes.POINTER(ctype))


# ---------------------------------------------------------------------------
# Functions with the C names (argument marshalling only)
# ---------------------------------------------------------------------------

def ising_word_rows(L):
    return int(_lib.load().ising_word_rows(int(L)))


def ising_required_bytes(L):
    return int(_lib.load().ising_required_bytes(int(L)))


def ising_thresholds(T):
    t4, t8 = ctypes.c_uint32(), ctypes.c_uint32()
    _check(_lib.load().ising_thresholds(float(T), ctypes.byref(t4), ctypes.byref(t8)))
    return int(t4.value), int(t8.value)


def ising_version():
    return _lib.load().ising_version().decode()


def ising_last_error():
    return _lib.load().ising_last_error().decode()


def ising_create(L, seed, init, stream=None):
    h = ctypes.c_void_p()
    _check(_lib.load().ising_create(int(L), int(seed), int(init), _stream(stream), ctypes.byref(h)))
    return h


def ising_create_in(L, seed, init, dev_words, nbytes, stream=None):
    h = ctypes.c_void_p()
    _check(_lib.load().ising_create_in(int(L), int(seed), int(init), _ptr(dev_words), int(nbytes), _stream(stream),
                                       ctypes.byref(h)))
    return h


def ising_reset(h, seed, init):
    _check(_lib.load().ising_reset(h, int(seed), int(init)))


def ising_destroy(h):
    _check(_lib.load().ising_destroy(h))


def ising_sweep(h, T, n_sweeps):
    _check(_lib.load().ising_sweep(h, float(T), int(n_sweeps)))


def ising_sweep_measure(h, T, n_sweeps, every, dev_E, dev_M):
    _check(_lib.load().ising_sweep_measure(h, float(T), int(n_sweeps), int(every), _ptr(dev_E), _ptr(dev_M)))


def ising_sweep_moments(h, T, n_sweeps, every, dev_acc):
    """dev_acc: device memory of one ising_moments (e.g. torch.zeros(10, dtype=torch.int64, device='cuda'))."""
    _check(_lib.load().ising_sweep_moments(h, float(T), int(n_sweeps), int(every), _ptr(dev_acc)))


def ising_scan(h, T, therm, meas, every):
    """Heating/cooling scan over the temperatures T (lattice carried over);
    one moments dict (exact Python ints) per temperature."""
    T_, pT = _arr(T, ctypes.c_double)
    out = (Moments * max(1, len(T_)))()
    _check(_lib.load().ising_scan(h, len(T_), pT, int(therm), int(meas), int(every), out))
    return [out[i].as_dict() for i in range(len(T_))]


def moments_of(acc):
    """Moments dict of a device accumulator filled by ising_sweep_moments."""
    raw = acc.detach().cpu().contiguous().numpy().tobytes() if hasattr(acc, "detach") else bytes(acc)
    return Moments.from_buffer_copy(raw[:ctypes.sizeof(Moments)]).as_dict()


def _moments_struct(m):
    if isinstance(m, Moments):
        return m
    out = Moments()
    out.n_samples, out.sum_E, out.sum_absM = int(m["n_samples"]), int(m["sum_E"]), int(m["sum_absM"])
    for name, limbs in (("sum_E2", 2), ("sum_M2", 2), ("sum_M4", 3)):
        v = int(m[name])
        for j in range(limbs):
            getattr(out, name)[j] = (v >> (64 * j)) & 0xFFFFFFFFFFFFFFFF
    return out


def ising_thermodynamics(m, L, T):
    """Per-spin e, c, |m|, chi, Binder cumulant of one moments dict (host arithmetic in the library)."""
    out = Thermo()
    _check(_lib.load().ising_thermodynamics(ctypes.byref(_moments_struct(m)), int(L), float(T), ctypes.byref(out)))
    return out.as_dict()


def ising_random_iterations(h, T, strip_cols, n_iterations, every=0, dev_E=None, dev_M=None, dev_acc=None):
    _check(_lib.load().ising_random_iterations(h, float(T), int(strip_cols), int(n_iterations), int(every),
                                               _ptr(dev_E), _ptr(dev_M), _ptr(dev_acc)))


def ising_observables(h):
    E, M = ctypes.c_int64(), ctypes.c_int64()
    _check(_lib.load().ising_observables(h, ctypes.byref(E), ctypes.byref(M)))
    return int(E.value), int(M.value)


def ising_get_spins(h, L):
    out = np.empty((L, L), dtype=np.uint8)
    _check(_lib.load().ising_get_spins(h, _ptr(out)))
    return out


def ising_get_spins_region(h, r0, c0, nrows, ncols):
    out = np.empty((nrows, ncols), dtype=np.uint8)
    _check(_lib.load().ising_get_spins_region(h, int(r0), int(c0), int(nrows), int(ncols), _ptr(out)))
    return out


def ising_set_spins(h, spins):
    s = np.ascontiguousarray(spins, dtype=np.uint8)
    _check(_lib.load().ising_set_spins(h, _ptr(s)))


def ising_get_sweep_count(h):
    t = ctypes.c_uint64()
    _check(_lib.load().ising_get_sweep_count(h, ctypes.byref(t)))
    return int(t.value)


def ising_set_sweep_count(h, t):
    _check(_lib.load().ising_set_sweep_count(h, int(t)))


def ising_words(h):
    p, n = ctypes.c_void_p(), ctypes.c_size_t()
    _check(_lib.load().ising_words(h, ctypes.byref(p), ctypes.byref(n)))
    return int(p.value or 0), int(n.value)


def ising_set_plan(h, words_per_thread, block):
    _check(_lib.load().ising_set_plan(h, int(words_per_thread), int(block)))


def ising_get_plan(h):
    w, b = ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.load().ising_get_plan(h, ctypes.byref(w), ctypes.byref(b)))
    return int(w.value), int(b.value)


def ising_autotune(h, T):
    ms = ctypes.c_double()
    _check(_lib.load().ising_autotune(h, float(T), ctypes.byref(ms)))
    return float(ms.value)


def ising_set_tiling(h, sweeps_per_launch, tile_cols=0, block=256):
    _check(_lib.load().ising_set_tiling(h, int(sweeps_per_launch), int(tile_cols), int(block)))


def ising_get_tiling(h):
    k, c, b = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.load().ising_get_tiling(h, ctypes.byref(k), ctypes.byref(c), ctypes.byref(b)))
    return int(k.value), int(c.value), int(b.value)


def ising_set_resident_tiles(h, tile_cols, block=512, max_sweeps=1000):
    _check(_lib.load().ising_set_resident_tiles(h, int(tile_cols), int(block), int(max_sweeps)))


def ising_set_resident_wait(h, ticks):
    _check(_lib.load().ising_set_resident_wait(h, int(ticks)))


def ising_get_resident_tiles(h):
    c, b, k = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.load().ising_get_resident_tiles(h, ctypes.byref(c), ctypes.byref(b), ctypes.byref(k)))
    return int(c.value), int(b.value), int(k.value)


def ising_sweep_measure_static(dev_words, nbytes, L, seed, t0, T, n_sweeps, every, dev_E, dev_M, stream=None):
    _check(_lib.load().ising_sweep_measure_static(_ptr(dev_words), int(nbytes), int(L), int(seed), int(t0), float(T),
                                                  int(n_sweeps), int(every), _ptr(dev_E), _ptr(dev_M),
                                                  _stream(stream)))


def ising_synchronize(h):
    _check(_lib.load().ising_synchronize(h))


def ising_batch_create(Ls, seeds, inits, stream=None):
    Ls_, pL = _arr(Ls, ctypes.c_int32)
    seeds_, pS = _arr(seeds, ctypes.c_uint64)
    inits_, pI = _arr(inits, ctypes.c_int32)
    h = ctypes.c_void_p()
    _check(_lib.load().ising_batch_create(len(Ls_), pL, pS, pI, _stream(stream), ctypes.byref(h)))
    return h


def ising_batch_destroy(h):
    _check(_lib.load().ising_batch_destroy(h))


def ising_batch_sweep(h, T, n_sweeps, every=0, dev_E=None, dev_M=None):
    T_, pT = _arr(T, ctypes.c_double)
    _check(_lib.load().ising_batch_sweep(h, pT, int(n_sweeps), int(every), _ptr(dev_E), _ptr(dev_M)))


def ising_batch_results(h, n):
    outs = [np.zeros(n, dtype=np.int64) for _ in range(5)]
    ptrs = [o.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) for o in outs]
    _check(_lib.load().ising_batch_results(h, *ptrs))
    return dict(zip(("E", "M", "sum_E", "sum_absM", "n_samples"), outs))


def ising_batch_reset_sums(h):
    _check(_lib.load().ising_batch_reset_sums(h))


def ising_batch_moments(h, n):
    out = (Moments * n)()
    _check(_lib.load().ising_batch_moments(h, out))
    return [out[i].as_dict() for i in range(n)]


def ising_batch_scan(h, n, T, therm, meas, every):
    """T: (n_T, n) temperatures, row j for step j; returns n_T lists of n moments dicts."""
    T_ = np.ascontiguousarray(np.asarray(T, dtype=np.float64).reshape(-1, n))
    n_T = T_.shape[0]
    out = (Moments * max(1, n_T * n))()
    _check(_lib.load().ising_batch_scan(h, n_T, T_.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(therm),
                                        int(meas), int(every), out))
    return [[out[j * n + i].as_dict() for i in range(n)] for j in range(n_T)]


def ising_batch_get_spins(h, i, L):
    out = np.empty((L, L), dtype=np.uint8)
    _check(_lib.load().ising_batch_get_spins(h, int(i), _ptr(out)))
    return out


def ising_batch_get_spins_region(h, i, r0, c0, nrows, ncols):
    out = np.empty((nrows, ncols), dtype=np.uint8)
    _check(_lib.load().ising_batch_get_spins_region(h, int(i), int(r0), int(c0), int(nrows), int(ncols), _ptr(out)))
    return out


def ising_batch_get_sweep_count(h, i):
    t = ctypes.c_uint64()
    _check(_lib.load().ising_batch_get_sweep_count(h, int(i), ctypes.byref(t)))
    return int(t.value)


def ising_batch_check_plan(plan):
    p = plan if isinstance(plan, BatchPlan) else BatchPlan(**plan)
    _check(_lib.load().ising_batch_check_plan(ctypes.byref(p)))


def ising_batch_set_plan(h, plan):
    p = plan if isinstance(plan, BatchPlan) else BatchPlan(**plan)
    _check(_lib.load().ising_batch_set_plan(h, ctypes.byref(p)))


def ising_batch_get_plan(h):
    p = BatchPlan()
    _check(_lib.load().ising_batch_get_plan(h, ctypes.byref(p)))
    return p.as_dict()


def ising_batch_autotune(h, T, cache_path=None):
    T_, pT = _arr(T, ctypes.c_double)
    p = BatchPlan()
    _check(_lib.load().ising_batch_autotune(h, pT, cache_path.encode() if cache_path else None, ctypes.byref(p)))
    return p.as_dict()


REPLICAS = 21


def _temps21(T):
    return _arr(np.broadcast_to(np.asarray(T, dtype=np.float64), (REPLICAS,)), ctypes.c_double)


def ising_replicas_create(L, seed, init, stream=None):
    h = ctypes.c_void_p()
    _check(_lib.load().ising_replicas_create(int(L), int(seed), int(init), _stream(stream), ctypes.byref(h)))
    return h


def ising_replicas_destroy(h):
    _check(_lib.load().ising_replicas_destroy(h))


def ising_replicas_sweep(h, T, n_sweeps):
    T_, pT = _temps21(T)
    _check(_lib.load().ising_replicas_sweep(h, pT, int(n_sweeps)))


def ising_replicas_sweep_measure(h, T, n_sweeps, every, dev_E, dev_M):
    T_, pT = _temps21(T)
    _check(_lib.load().ising_replicas_sweep_measure(h, pT, int(n_sweeps), int(every), _ptr(dev_E), _ptr(dev_M)))


def ising_replicas_sweep_moments(h, T, n_sweeps, every, dev_acc):
    T_, pT = _temps21(T)
    _check(_lib.load().ising_replicas_sweep_moments(h, pT, int(n_sweeps), int(every), _ptr(dev_acc)))


def ising_replicas_observables(h):
    E = np.zeros(REPLICAS, dtype=np.int64)
    M = np.zeros(REPLICAS, dtype=np.int64)
    _check(_lib.load().ising_replicas_observables(h, E.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                                  M.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
    return E, M


def ising_replicas_get_spins(h, k, L):
    out = np.empty((L, L), dtype=np.uint8)
    _check(_lib.load().ising_replicas_get_spins(h, int(k), _ptr(out)))
    return out


def ising_replicas_get_sweep_count(h):
    t = ctypes.c_uint64()
    _check(_lib.load().ising_replicas_get_sweep_count(h, ctypes.byref(t)))
    return int(t.value)


def ising_replicas_set_plan(h, words_per_thread):
    _check(_lib.load().ising_replicas_set_plan(h, int(words_per_thread)))


def ising_server_create(hbm_budget, max_slots, quantum_sweeps, stream=None):
    h = ctypes.c_void_p()
    _check(_lib.load().ising_server_create(int(hbm_budget), int(max_slots), int(quantum_sweeps), _stream(stream),
                                           ctypes.byref(h)))
    return h


def ising_server_submit(h, req_id, L, T, sweeps, seed, init):
    _check(_lib.load().ising_server_submit(h, int(req_id), int(L), float(T), int(sweeps), int(seed), int(init)))


def ising_server_step(h):
    a = ctypes.c_int32()
    _check(_lib.load().ising_server_step(h, ctypes.byref(a)))
    return int(a.value)


def ising_server_poll(h, cap=4096):
    buf = (Result * cap)()
    n = ctypes.c_int32()
    _check(_lib.load().ising_server_poll(h, buf, int(cap), ctypes.byref(n)))
    out = []
    for i in range(n.value):
        r = buf[i]
        out.append({k: getattr(r, k) for k, _ in Result._fields_})
    return out


def ising_server_stats(h):
    q, r, f, b = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_size_t()
    _check(_lib.load().ising_server_stats(h, ctypes.byref(q), ctypes.byref(r), ctypes.byref(f), ctypes.byref(b)))
    return {"queued": q.value, "resident": r.value, "finished": f.value, "bytes_in_use": b.value}


def ising_server_destroy(h):
    _check(_lib.load().ising_server_destroy(h))


# ---------------------------------------------------------------------------
# Convenience classes
# ---------------------------------------------------------------------------

class Lattice:
    """One L x L lattice whose packed words live in a torch CUDA tensor."""

    def __init__(self, L, seed, hot=True, stream=None, device="cuda"):
        import torch

        self.L = int(L)
        self.seed = int(seed)
        nbytes = ising_required_bytes(self.L)
        if nbytes == 0:
            raise IsingError(ISING_EINVAL, f"invalid lattice size L={L}")
        self.stream = stream
        self._order = _Ordering(stream)
        self.words = torch.empty(nbytes // 8, dtype=torch.int64, device=device)
        self._order.before()  # the block may still be in use by work on torch's stream
        self.handle = ising_create_in(self.L, self.seed, ISING_HOT if hot else ISING_COLD, self.words, nbytes, stream)
        self._order.after(self.words)

    def reset(self, seed=None, hot=True):
        if seed is not None:
            self.seed = int(seed)
        ising_reset(self.handle, self.seed, ISING_HOT if hot else ISING_COLD)
        return self

    def sweep(self, T, n):
        ising_sweep(self.handle, T, n)
        return self

    def sweep_measure(self, T, n, every):
        """Returns device int64 tensors (E, M) of n // every samples."""
        import torch

        k = int(n) // int(every)
        E = torch.empty(max(k, 1), dtype=torch.int64, device=self.words.device)
        M = torch.empty(max(k, 1), dtype=torch.int64, device=self.words.device)
        self._order.before()
        ising_sweep_measure(self.handle, T, n, every, E, M)
        self._order.after(E, M)
        return E[:k], M[:k]

    def sweep_moments(self, T, n, every, acc=None):
        """Adds the samples' moments to `acc` (a device int64 tensor of 10, zeroed if None) and returns it."""
        import torch

        if acc is None:
            acc = torch.zeros(10, dtype=torch.int64, device=self.words.device)
        self._order.before()
        ising_sweep_moments(self.handle, T, n, every, acc)
        self._order.after(acc)
        return acc

    def scan(self, T, therm, meas, every=1):
        return ising_scan(self.handle, T, therm, meas, every)

    def random_iterations(self, T, strip_cols, n, every=0, acc=None):
        """The paper's strip dynamics; with every > 0 returns device (E, M)
        series of n // every samples (and adds them to `acc` if given)."""
        import torch

        if every > 0:
            k = int(n) // int(every)
            E = torch.empty(max(k, 1), dtype=torch.int64, device=self.words.device)
            M = torch.empty(max(k, 1), dtype=torch.int64, device=self.words.device)
            self._order.before()
            ising_random_iterations(self.handle, T, strip_cols, n, every, E, M, acc)
            self._order.after(E, M, acc)
            return E[:k], M[:k]
        ising_random_iterations(self.handle, T, strip_cols, n, 0)
        return None

    def observables(self):
        return ising_observables(self.handle)

    def spins(self):
        return ising_get_spins(self.handle, self.L)

    def region(self, r0, c0, nrows, ncols):
        return ising_get_spins_region(self.handle, r0, c0, nrows, ncols)

    def set_spins(self, s):
        ising_set_spins(self.handle, s)

    @property
    def t(self):
        return ising_get_sweep_count(self.handle)

    @t.setter
    def t(self, value):
        ising_set_sweep_count(self.handle, value)

    def set_plan(self, words_per_thread, block):
        ising_set_plan(self.handle, words_per_thread, block)

    def plan(self):
        return ising_get_plan(self.handle)

    def set_tiling(self, sweeps_per_launch, tile_cols=0, block=256):
        ising_set_tiling(self.handle, sweeps_per_launch, tile_cols, block)

    def tiling(self):
        return ising_get_tiling(self.handle)

    def set_resident_tiles(self, tile_cols, block=512, max_sweeps=1000):
        ising_set_resident_tiles(self.handle, tile_cols, block, max_sweeps)

    def resident_tiles(self):
        return ising_get_resident_tiles(self.handle)

    def set_resident_wait(self, ticks):
        ising_set_resident_wait(self.handle, ticks)

    def autotune(self, T):
        return ising_autotune(self.handle, T)

    def synchronize(self):
        ising_synchronize(self.handle)

    def close(self):
        if getattr(self, "handle", None) is not None:
            ising_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many lattices of mixed L advanced together (one graph replay per chunk)."""

    def __init__(self, Ls, seeds, hot=True, stream=None):
        self.Ls = [int(x) for x in Ls]
        hots = [hot] * len(self.Ls) if isinstance(hot, bool) else list(hot)
        inits = [ISING_HOT if h else ISING_COLD for h in hots]
        self._order = _Ordering(stream)
        self.handle = ising_batch_create(self.Ls, seeds, inits, stream)

    def __len__(self):
        return len(self.Ls)

    def sweep(self, T, n, every=0, series=False):
        import torch

        T = np.broadcast_to(np.asarray(T, dtype=np.float64), (len(self.Ls),))
        if series and every > 0:
            k = int(n) // int(every)
            E = torch.empty(max(1, len(self.Ls) * k), dtype=torch.int64, device="cuda")
            M = torch.empty_like(E)
            self._order.before()
            ising_batch_sweep(self.handle, T, n, every, E, M)
            self._order.after(E, M)
            return E[: len(self.Ls) * k].view(len(self.Ls), k), M[: len(self.Ls) * k].view(len(self.Ls), k)
        ising_batch_sweep(self.handle, T, n, every)
        return None

    def results(self):
        return ising_batch_results(self.handle, len(self.Ls))

    def reset_sums(self):
        ising_batch_reset_sums(self.handle)

    def moments(self):
        return ising_batch_moments(self.handle, len(self.Ls))

    def scan(self, T, therm, meas, every=1):
        """T: one temperature per step (shared by all lattices) or an (n_T, n) array."""
        T = np.asarray(T, dtype=np.float64)
        if T.ndim == 1:
            T = np.repeat(T[:, None], len(self.Ls), axis=1)
        return ising_batch_scan(self.handle, len(self.Ls), T, therm, meas, every)

    def spins(self, i):
        return ising_batch_get_spins(self.handle, i, self.Ls[i])

    def region(self, i, r0, c0, nrows, ncols):
        return ising_batch_get_spins_region(self.handle, i, r0, c0, nrows, ncols)

    def sweep_count(self, i):
        return ising_batch_get_sweep_count(self.handle, i)

    def set_plan(self, **plan):
        ising_batch_set_plan(self.handle, plan)

    def plan(self):
        return ising_batch_get_plan(self.handle)

    def autotune(self, T, cache_path=None):
        T = np.broadcast_to(np.asarray(T, dtype=np.float64), (len(self.Ls),))
        return ising_batch_autotune(self.handle, T, cache_path)

    def close(self):
        if getattr(self, "handle", None) is not None:
            ising_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Replicas:
    """21 independent L x L lattices packed field by field into one word lattice."""

    def __init__(self, L, seed, hot=True, stream=None):
        self.L = int(L)
        self._order = _Ordering(stream)
        self.handle = ising_replicas_create(self.L, seed, ISING_HOT if hot else ISING_COLD, stream)

    def sweep(self, T, n):
        ising_replicas_sweep(self.handle, T, n)
        return self

    def sweep_measure(self, T, n, every):
        """Device int64 tensors (E, M) of shape (n // every, 21)."""
        import torch

        k = int(n) // int(every)
        E = torch.empty(max(k, 1) * REPLICAS, dtype=torch.int64, device="cuda")
        M = torch.empty_like(E)
        self._order.before()
        ising_replicas_sweep_measure(self.handle, T, n, every, E, M)
        self._order.after(E, M)
        return E[: k * REPLICAS].view(k, REPLICAS), M[: k * REPLICAS].view(k, REPLICAS)

    def sweep_moments(self, T, n, every, acc=None):
        """Adds the samples to `acc` (device int64 tensor of 21 x 10, zeroed if None); returns it."""
        import torch

        if acc is None:
            acc = torch.zeros(REPLICAS * 10, dtype=torch.int64, device="cuda")
        self._order.before()
        ising_replicas_sweep_moments(self.handle, T, n, every, acc)
        self._order.after(acc)
        return acc

    def moments(self, acc):
        raw = acc.detach().cpu().contiguous().numpy().tobytes()
        size = ctypes.sizeof(Moments)
        return [Moments.from_buffer_copy(raw[k * size:(k + 1) * size]).as_dict() for k in range(REPLICAS)]

    def observables(self):
        return ising_replicas_observables(self.handle)

    def spins(self, k):
        return ising_replicas_get_spins(self.handle, k, self.L)

    @property
    def t(self):
        return ising_replicas_get_sweep_count(self.handle)

    def set_plan(self, words_per_thread):
        ising_replicas_set_plan(self.handle, words_per_thread)

    def close(self):
        if getattr(self, "handle", None) is not None:
            ising_replicas_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching request server."""

    def __init__(self, hbm_budget, max_slots=4096, quantum_sweeps=100, stream=None):
        self.handle = ising_server_create(hbm_budget, max_slots, quantum_sweeps, stream)

    def submit(self, req_id, L, T, sweeps, seed=None, hot=True):
        ising_server_submit(self.handle, req_id, L, T, sweeps, req_id if seed is None else seed,
                            ISING_HOT if hot else ISING_COLD)

    def step(self):
        return ising_server_step(self.handle)

    def poll(self, cap=4096):
        return ising_server_poll(self.handle, cap)

    def stats(self):
        return ising_server_stats(self.handle)

    def close(self):
        if getattr(self, "handle", None) is not None:
            ising_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
