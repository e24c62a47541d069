"""ctypes binding of libspr.so (include/spr.h): argument marshalling only.

Every computation runs in the HIP library.  Host arrays are NumPy arrays; device
arrays are torch tensors on the context's device (passed by data pointer with
SPR_DEVICE_PTRS).  Loading fails loudly when the library has not been built.
"""

import atexit
import ctypes as C
import os
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspr.so")

SPR_OK = 0
STATUS = {0: "SPR_OK", -1: "SPR_E_INVALID_ARG", -2: "SPR_E_UNSUPPORTED_SIZE", -3: "SPR_E_OOM",
          -4: "SPR_E_HIP", -5: "SPR_E_NOT_READY", -6: "SPR_E_BUSY", -7: "SPR_E_NUMERIC",
          -8: "SPR_E_ADMISSION"}
STATUS_NOT_READY = -5
E_BUSY = -6
E_ADMISSION = -8

DEVICE_PTRS = 0x1
LAYOUT_FFT = 0x2
POP_MEMETIC = 0x4
READ_CHILDREN = 0x8
INIT_RANDOM_PHASE = 0x10
AMP_FP16 = 0x20

ITER_TRACE = 1
OP_ER, OP_HIO, OP_RAAR, OP_SHRINKWRAP, OP_SUPPORT_AREA, OP_GET_ERROR, OP_STATS, OP_CROSSOVER, OP_SELECT, OP_AVERAGE, \
    OP_MONITOR = range(1, 12)
ALG_HIO, ALG_RAAR = 1, 2
AREA_BEST, AREA_EVAL, AREA_ABS = 0, 1, 2
SCOPE_ALL, SCOPE_PARENTS, SCOPE_CHILDREN = 0, 1, 2


class SprError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Op(C.Structure):
    _fields_ = [("kind", C.c_int32), ("count", C.c_int32), ("scope", C.c_int32), ("which", C.c_int32),
                ("gen", C.c_int32), ("gens", C.c_int32), ("t_min", C.c_int32), ("t_max", C.c_int32),
                ("beta", C.c_double), ("chi", C.c_double), ("sigma", C.c_double), ("tau", C.c_double),
                ("alpha", C.c_double), ("c_p", C.c_double), ("c_w", C.c_double), ("c_a", C.c_double)]


class PlainParams(C.Structure):
    _fields_ = [("alg", C.c_int32), ("G", C.c_int32), ("j", C.c_int32), ("j_er", C.c_int32),
                ("j_end", C.c_int32), ("beta", C.c_double), ("chi", C.c_double), ("sigma", C.c_double),
                ("sigma_end", C.c_double), ("tau", C.c_double), ("tau_end", C.c_double)]


class MprParams(C.Structure):
    _fields_ = [("alg", C.c_int32), ("G", C.c_int32), ("R", C.c_int32), ("j", C.c_int32),
                ("j_er", C.c_int32), ("j_end", C.c_int32), ("j_eval", C.c_int32), ("t_min", C.c_int32),
                ("t_max", C.c_int32), ("gen_first", C.c_int32), ("gen_count", C.c_int32),
                ("init_error", C.c_int32), ("beta", C.c_double), ("chi", C.c_double),
                ("sigma", C.c_double), ("sigma_end", C.c_double), ("tau", C.c_double),
                ("tau_end", C.c_double), ("c_p", C.c_double), ("c_w", C.c_double), ("c_a", C.c_double),
                ("monitor", C.c_int32), ("pad", C.c_int32)]


class GenStats(C.Structure):
    _fields_ = [("gen", C.c_int32), ("best", C.c_int32), ("alpha_best", C.c_int32),
                ("alpha_all", C.c_int32), ("alpha_eval", C.c_double), ("err_best", C.c_double),
                ("err_mean", C.c_double), ("err_worst", C.c_double), ("replaced", C.c_int32),
                ("pad", C.c_int32)]


class XoverInfo(C.Structure):
    _fields_ = [("a", C.c_int32), ("b", C.c_int32), ("c", C.c_int32), ("tx", C.c_int32),
                ("ty", C.c_int32), ("sx", C.c_int32), ("sy", C.c_int32), ("rot", C.c_int32),
                ("dr", C.c_int32 * 3), ("dc", C.c_int32 * 3), ("twin", C.c_int32 * 3),
                ("phase", (C.c_float * 2) * 3), ("peak", (C.c_float * 2) * 3)]


class Monitor(C.Structure):
    _fields_ = [("gen", C.c_int32), ("P", C.c_int32), ("err_best", C.c_double), ("err_median", C.c_double),
                ("err_worst", C.c_double), ("err_mean", C.c_double), ("gamma_mean", C.c_double),
                ("sum_mean", C.c_double), ("sum_rel_std", C.c_double), ("gamma_avg", C.c_double),
                ("err_avg", C.c_double), ("has_avg", C.c_int32), ("pad", C.c_int32)]


class SphereParams(C.Structure):
    _fields_ = [("sigma_init", C.c_double), ("n_init", C.c_int32), ("set_support", C.c_int32),
                ("diam_min", C.c_double), ("diam_max", C.c_double), ("phase_min", C.c_double),
                ("phase_max", C.c_double), ("gamma", C.c_double)]


class ServerCfg(C.Structure):
    _fields_ = [("hbm_budget", C.c_uint64), ("max_shots", C.c_int32), ("P", C.c_int32),
                ("sched", C.c_void_p), ("flags", C.c_uint32), ("max_inflight", C.c_int32),
                ("max_queue", C.c_uint64), ("sim_bytes_per_s", C.c_double), ("sim_launch_s", C.c_double)]


class ShotDesc(C.Structure):
    _fields_ = [("n", C.c_int32), ("amp", C.c_void_p), ("mask", C.c_void_p), ("supp0", C.c_void_p),
                ("supp_per_member", C.c_int32), ("flags", C.c_uint32), ("rho0", C.c_void_p),
                ("seed", C.c_uint64), ("arrival", C.c_double), ("bound_eta", C.c_double),
                ("bound_max_unknown", C.c_double), ("saturated", C.c_void_p), ("bound_max_saturated", C.c_double)]


class Result(C.Structure):
    _fields_ = [("rho", C.c_void_p), ("supp", C.c_void_p), ("err", C.c_void_p), ("n", C.c_int32),
                ("P", C.c_int32), ("members", C.c_int32), ("best", C.c_int32), ("t_arrival", C.c_double),
                ("t_admit", C.c_double), ("t_finish", C.c_double), ("status", C.c_int32), ("pad", C.c_int32)]


class ServerStats(C.Structure):
    _fields_ = [("now", C.c_double), ("queued", C.c_int64), ("active", C.c_int64), ("finishing", C.c_int64),
                ("done", C.c_int64), ("admitted", C.c_int64), ("completed", C.c_int64), ("ticks", C.c_int64),
                ("launches", C.c_int64), ("max_active", C.c_int64), ("bytes_capacity", C.c_uint64),
                ("bytes_in_use", C.c_uint64), ("bytes_peak", C.c_uint64)]


class TuneResult(C.Structure):
    _fields_ = [("n", C.c_int32), ("variant", C.c_int32), ("chunk_members", C.c_int32), ("candidates", C.c_int32),
                ("member_iterations_per_s", C.c_double), ("cand_variant", C.c_int32 * 16),
                ("cand_chunk", C.c_int32 * 16), ("cand_rate", C.c_double * 16)]


SERVER_MANUAL = 0x1
SERVER_ALL_MEMBERS = 0x2
SERVER_SHORTEST_FIRST = 0x4

EXPORTS = ["spr_ctx_create", "spr_ctx_destroy", "spr_ctx_last_error", "spr_supported_size",
           "spr_shot_create", "spr_shot_destroy", "spr_pop_create", "spr_pop_destroy", "spr_pop_write",
           "spr_sched_create", "spr_sched_plain", "spr_sched_mpr", "spr_sched_destroy", "spr_sched_ops",
           "spr_run", "spr_sync", "spr_read", "spr_read_stats", "spr_read_xover", "spr_fft2", "spr_fft2_noalloc",
           "spr_timing_enable", "spr_timing_sample", "spr_timing_read", "spr_ctx_set_cache_budget", "spr_run_batch",
           "spr_read_member", "spr_read_average", "spr_read_monitor", "spr_read_trace", "spr_pop_init_spheres", "spr_shot_set_bounds", "spr_shot_set_bounds_sat", "spr_size_variants", "spr_ctx_autotune", "spr_ctx_set_variant",
           "spr_ctx_get_tuning", "spr_graph_create", "spr_graph_create_batch", "spr_graph_launch",
           "spr_graph_destroy", "spr_server_create", "spr_server_submit", "spr_server_poll", "spr_server_step", "spr_server_drain",
           "spr_server_stats_get", "spr_server_last_error", "spr_server_destroy"]

KERNEL_ROW_INGEST, KERNEL_COL_PROJ, KERNEL_ROW_UPDATE_ER, KERNEL_ROW_UPDATE_IA = range(4)
KERNEL_NAMES = {0: "k_row_ingest", 1: "k_col_proj", 2: "k_row_update(ER)", 3: "k_row_update(HIO/RAAR)"}

_lib = None


def _proto(lib):
    vp, i32, u32, u64 = C.c_void_p, C.c_int32, C.c_uint32, C.c_uint64
    pp = C.POINTER(C.c_void_p)
    sig = {
        "spr_ctx_create": (i32, [i32, pp]),
        "spr_ctx_destroy": (None, [vp]),
        "spr_ctx_last_error": (C.c_char_p, [vp]),
        "spr_supported_size": (i32, [i32]),
        "spr_shot_create": (i32, [vp, i32, vp, vp, u32, pp]),
        "spr_shot_destroy": (i32, [vp]),
        "spr_pop_create": (i32, [vp, i32, vp, vp, i32, u32, u64, i32, pp]),
        "spr_pop_destroy": (i32, [vp]),
        "spr_pop_write": (i32, [vp, vp, vp, vp, u32]),
        "spr_sched_create": (i32, [vp, C.POINTER(Op), i32, pp]),
        "spr_sched_plain": (i32, [vp, C.POINTER(PlainParams), pp]),
        "spr_sched_mpr": (i32, [vp, C.POINTER(MprParams), pp]),
        "spr_sched_destroy": (i32, [vp]),
        "spr_sched_ops": (i32, [vp, C.POINTER(Op), i32, C.POINTER(i32)]),
        "spr_run": (i32, [vp, vp, vp]),
        "spr_sync": (i32, [vp]),
        "spr_read": (i32, [vp, vp, vp, vp, u32]),
        "spr_read_stats": (i32, [vp, C.POINTER(GenStats), i32, C.POINTER(i32)]),
        "spr_read_xover": (i32, [vp, C.POINTER(XoverInfo), i32]),
        "spr_fft2": (i32, [vp, i32, i32, vp, vp, i32, vp]),
        "spr_fft2_noalloc": (i32, [vp, i32, i32, vp, vp, i32, vp]),
        "spr_timing_enable": (i32, [vp, i32]),
        "spr_timing_sample": (i32, [vp, i32]),
        "spr_timing_read": (i32, [vp, i32, C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
        "spr_ctx_set_cache_budget": (i32, [vp, C.c_uint64]),
        "spr_run_batch": (i32, [vp, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), i32, vp]),
        "spr_read_member": (i32, [vp, i32, vp, vp, u32]),
        "spr_read_average": (i32, [vp, vp, vp, vp, u32]),
        "spr_read_monitor": (i32, [vp, C.POINTER(Monitor), i32, C.POINTER(i32)]),
        "spr_read_trace": (i32, [vp, vp, i32, C.POINTER(i32), C.POINTER(i32)]),
        "spr_pop_init_spheres": (i32, [vp, C.POINTER(SphereParams)]),
        "spr_shot_set_bounds": (i32, [vp, C.c_double, C.c_double, C.POINTER(i32)]),
        "spr_shot_set_bounds_sat": (i32, [vp, C.c_double, C.c_double, vp, C.c_double, C.c_uint32,
                                          C.POINTER(i32)]),
        "spr_size_variants": (i32, [i32]),
        "spr_ctx_autotune": (i32, [vp, i32, i32, C.POINTER(TuneResult)]),
        "spr_ctx_set_variant": (i32, [vp, i32, i32, i32]),
        "spr_ctx_get_tuning": (i32, [vp, i32, C.POINTER(i32), C.POINTER(i32)]),
        "spr_graph_create": (i32, [vp, vp, pp]),
        "spr_graph_create_batch": (i32, [vp, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), i32, pp]),
        "spr_graph_launch": (i32, [vp, vp]),
        "spr_graph_destroy": (i32, [vp]),
        "spr_server_create": (i32, [vp, C.POINTER(ServerCfg), pp]),
        "spr_server_submit": (i32, [vp, C.POINTER(ShotDesc), C.POINTER(C.c_uint64)]),
        "spr_server_poll": (i32, [vp, C.c_uint64, C.POINTER(Result)]),
        "spr_server_step": (i32, [vp, C.POINTER(C.c_int64)]),
        "spr_server_drain": (i32, [vp, C.c_double]),
        "spr_server_stats_get": (i32, [vp, C.POINTER(ServerStats)]),
        "spr_server_last_error": (C.c_char_p, [vp]),
        "spr_server_destroy": (i32, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args


def load():
    """Load libspr.so (raises if it has not been built).

    A process must hold one HIP runtime.  PyTorch ships its own libamdhip64
    with the same soname as the system one; importing torch first makes
    libspr.so bind to that copy, so torch streams and device pointers are valid
    in the library.  Without torch the system runtime is used.
    """
    global _lib
    if _lib is None:
        try:
            import torch  # noqa: F401  (loads the process-wide HIP runtime first)
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run python -m paper_2409_07413_amd.build)")
        lib = C.CDLL(LIB_PATH)
        _proto(lib)
        _lib = lib
    return _lib


def _ptr(a):
    """(pointer, is_device) for a NumPy array or torch tensor (None -> null)."""
    if a is None:
        return None, False
    if isinstance(a, np.ndarray):
        if not a.flags["C_CONTIGUOUS"]:
            raise ValueError("arrays must be C-contiguous")
        return a.ctypes.data, False
    if hasattr(a, "data_ptr"):
        if not a.is_contiguous():
            raise ValueError("tensors must be contiguous")
        return a.data_ptr(), a.is_cuda
    raise TypeError(f"unsupported array type {type(a)}")


def check(st, ctx_handle=None):
    """Raise SprError for a non-zero status, with the context's message."""
    if st != SPR_OK:
        msg = ""
        if ctx_handle:
            raw = load().spr_ctx_last_error(ctx_handle)
            msg = raw.decode() if raw else ""
        raise SprError(st, msg)


def sched_ops(ops, ctx=None):
    """Schedule from a list of Op (host-only call)."""
    lib = load()
    arr = (Op * len(ops))(*ops)
    h = C.c_void_p()
    check(lib.spr_sched_create(ctx.h if ctx else None, arr, len(ops), C.byref(h)), ctx.h if ctx else None)
    return Schedule(ctx, h)


def sched_plain(ctx=None, **kw):
    """Alg. randomsearch/normalimprove schedule (host-only call)."""
    lib = load()
    prm = PlainParams(**kw)
    h = C.c_void_p()
    check(lib.spr_sched_plain(ctx.h if ctx else None, C.byref(prm), C.byref(h)), ctx.h if ctx else None)
    return Schedule(ctx, h)


def sched_mpr(ctx=None, **kw):
    """Alg. mpr schedule (host-only call)."""
    lib = load()
    prm = MprParams(**kw)
    h = C.c_void_p()
    check(lib.spr_sched_mpr(ctx.h if ctx else None, C.byref(prm), C.byref(h)), ctx.h if ctx else None)
    return Schedule(ctx, h)


def _stream_ptr(stream):
    if stream is None:
        return None
    return getattr(stream, "cuda_stream", stream)


_live_contexts = weakref.WeakSet()


@atexit.register
def _close_all():
    """Release every library handle before the interpreter tears down, so no
    finaliser calls into the HIP runtime during the final collection."""
    for ctx in list(_live_contexts):
        try:
            ctx.close()
        except Exception:
            pass


class Context:
    def __init__(self, device=0):
        self.lib = load()
        self._pops = weakref.WeakSet()
        self._shots = weakref.WeakSet()
        self._servers = weakref.WeakSet()
        self._graphs = weakref.WeakSet()
        h = C.c_void_p()
        self._check(self.lib.spr_ctx_create(int(device), C.byref(h)), ctx=None)
        self.h = h
        _live_contexts.add(self)

    def _check(self, st, ctx="self"):
        check(st, self.h if ctx == "self" else ctx)

    def close(self):
        """Destroy the context, closing its populations and shots first."""
        if getattr(self, "h", None):
            for sv in list(getattr(self, "_servers", ())):
                sv.close()
            for g in list(getattr(self, "_graphs", ())):
                g.close()
            for p in list(getattr(self, "_pops", ())):
                p.close()
            for sh in list(getattr(self, "_shots", ())):
                try:
                    sh.close()
                except SprError:
                    pass
            self.lib.spr_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_cache_budget(self, nbytes):
        """Member-chunk budget of iteration runs in bytes (0 = no chunks)."""
        self._check(self.lib.spr_ctx_set_cache_budget(self.h, int(nbytes)))

    def run_batch(self, pops, scheds, stream=None):
        """Run scheds[i] on pops[i]; same-size populations share every launch."""
        n = len(pops)
        ph = (C.c_void_p * n)(*[p.h.value if isinstance(p.h, C.c_void_p) else p.h for p in pops])
        sh = (C.c_void_p * n)(*[s.h.value if isinstance(s.h, C.c_void_p) else s.h for s in scheds])
        self._check(self.lib.spr_run_batch(self.h, ph, sh, n, _stream_ptr(stream)))

    def autotune(self, n, members):
        """Time every kernel variant and member chunk of size n; keep the fastest."""
        r = TuneResult()
        self._check(self.lib.spr_ctx_autotune(self.h, int(n), int(members), C.byref(r)))
        cands = [{"variant": r.cand_variant[i], "chunk_members": r.cand_chunk[i],
                  "member_iterations_per_s": r.cand_rate[i]} for i in range(r.candidates)]
        return {"n": r.n, "variant": r.variant, "chunk_members": r.chunk_members,
                "member_iterations_per_s": r.member_iterations_per_s, "candidates": cands}

    def set_variant(self, n, variant, chunk_members=0):
        self._check(self.lib.spr_ctx_set_variant(self.h, int(n), int(variant), int(chunk_members)))

    def tuning(self, n):
        v, c = C.c_int32(), C.c_int32()
        self._check(self.lib.spr_ctx_get_tuning(self.h, int(n), C.byref(v), C.byref(c)))
        return v.value, c.value

    def graph_batch(self, pops, scheds):
        """Capture a batch (as run_batch would run it) into a replayable graph."""
        n = len(pops)
        ph = (C.c_void_p * n)(*[p.h.value if isinstance(p.h, C.c_void_p) else p.h for p in pops])
        sh = (C.c_void_p * n)(*[s.h.value if isinstance(s.h, C.c_void_p) else s.h for s in scheds])
        h = C.c_void_p()
        self._check(self.lib.spr_graph_create_batch(self.h, ph, sh, n, C.byref(h)))
        return Graph(self, h, pops)

    def supported(self, n):
        return bool(self.lib.spr_supported_size(int(n)))

    def shot(self, amp, mask, fft_order=False, fp16=False):
        """amp: N x N float32 (centred unless fft_order); mask: N x N uint8 (1 = measured).
        fp16: keep the modulus in FP16 on the device (power-of-two scaled)."""
        return Shot(self, amp, mask, fft_order, fp16)

    def sched_ops(self, ops):
        return sched_ops(ops, self)

    def sched_plain(self, **kw):
        return sched_plain(self, **kw)

    def sched_mpr(self, **kw):
        return sched_mpr(self, **kw)

    def fft2(self, x_in, x_out, inverse=False, stream=None):
        """Unitary 2D DFT of a batch of N x N complex64 device tensors.

        With stream=None the call is ordered with torch's work by device-wide
        synchronisation before and after (torch's default stream has the null
        handle, which the library reads as its own context stream).
        """
        n = x_in.shape[-1]
        batch = x_in.numel() // (n * n)
        pi, di = _ptr(x_in)
        po, do = _ptr(x_out)
        if not (di and do):
            raise ValueError("fft2 takes device tensors")
        sp = _stream_ptr(stream)
        if not sp:
            import torch
            torch.cuda.synchronize()
        self._check(self.lib.spr_fft2(self.h, n, batch, pi, po, 1 if inverse else 0, sp))
        if not sp:
            torch.cuda.synchronize()

    def fft2_noalloc(self, x_in, x_out, inverse=False, stream=None):
        """The same transform through the allocation-free entry point (its
        intermediate in the library's fixed device scratch array)."""
        n = x_in.shape[-1]
        batch = x_in.numel() // (n * n)
        pi, di = _ptr(x_in)
        po, do = _ptr(x_out)
        if not (di and do):
            raise ValueError("fft2_noalloc takes device tensors")
        sp = _stream_ptr(stream)
        if not sp:
            import torch
            torch.cuda.synchronize()
        self._check(self.lib.spr_fft2_noalloc(self.h, n, batch, pi, po, 1 if inverse else 0, sp))
        if not sp:
            torch.cuda.synchronize()


class Shot:
    def __init__(self, ctx, amp, mask, fft_order=False, fp16=False):
        self.ctx = ctx
        self.n = int(amp.shape[-1])
        pa, da = _ptr(amp)
        pm, dm = _ptr(mask)
        if da != dm:
            raise ValueError("amp and mask must both be host or both be device arrays")
        flags = (DEVICE_PTRS if da else 0) | (LAYOUT_FFT if fft_order else 0) | (AMP_FP16 if fp16 else 0)
        h = C.c_void_p()
        ctx._check(ctx.lib.spr_shot_create(ctx.h, self.n, pa, pm, flags, C.byref(h)))
        self.h = h
        self._keep = (amp, mask)
        self._fft_order = bool(fft_order)
        ctx._shots.add(self)

    def close(self):
        if getattr(self, "h", None):
            st = self.ctx.lib.spr_shot_destroy(self.h)
            self.ctx._check(st)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_bounds(self, eta=1.5, max_unknown=0.2, saturated=None, max_saturated=0.05):
        """Upper bounds on the unknown amplitudes from the radial profile; returns the bounded rings.
        `saturated` (N*N, the shot's layout, host or device): the saturation rules apply."""
        r = C.c_int32()
        if saturated is None:
            self.ctx._check(self.ctx.lib.spr_shot_set_bounds(self.h, float(eta), float(max_unknown), C.byref(r)))
            return r.value
        if isinstance(saturated, np.ndarray):
            saturated = np.ascontiguousarray(saturated, dtype=np.uint8)
        ps, ds = _ptr(saturated)
        flags = (DEVICE_PTRS if ds else 0) | (LAYOUT_FFT if self._fft_order else 0)
        self.ctx._check(self.ctx.lib.spr_shot_set_bounds_sat(self.h, float(eta), float(max_unknown), ps,
                                                             float(max_saturated), flags, C.byref(r)))
        return r.value

    def population(self, rho0, supp0, memetic=False, seed=0, gen_offset=0, P=None):
        """rho0 None: P members from the device-side random-phase start keyed by seed."""
        return Population(self, rho0, supp0, memetic, seed, gen_offset, P)


class Schedule:
    def __init__(self, ctx, h):
        self.ctx = ctx
        self.h = h

    def ops(self):
        lib = load()
        n = C.c_int32()
        check(lib.spr_sched_ops(self.h, None, 0, C.byref(n)))
        arr = (Op * n.value)()
        check(lib.spr_sched_ops(self.h, arr, n.value, C.byref(n)))
        return list(arr)

    def close(self):
        if getattr(self, "h", None):
            load().spr_sched_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Population:
    def __init__(self, shot, rho0, supp0, memetic, seed, gen_offset, P=None):
        self.shot = shot
        self.ctx = shot.ctx
        self.n = shot.n
        ps, ds = _ptr(supp0)
        flags = POP_MEMETIC if memetic else 0
        if rho0 is None:
            if P is None:
                raise ValueError("P is needed for the random-phase start")
            self.P = int(P)
            pr, dr = None, ds
            flags |= INIT_RANDOM_PHASE
        else:
            self.P = int(rho0.shape[0])
            pr, dr = _ptr(rho0)
        if dr != ds:
            raise ValueError("rho0 and supp0 must both be host or both be device arrays")
        per_member = 1 if supp0.ndim == 3 else 0
        flags |= DEVICE_PTRS if dr else 0
        h = C.c_void_p()
        self.ctx._check(self.ctx.lib.spr_pop_create(shot.h, self.P, pr, ps, per_member, flags,
                                                    int(seed) & 0xFFFFFFFFFFFFFFFF, int(gen_offset),
                                                    C.byref(h)))
        self.h = h
        self.ctx._pops.add(self)

    def close(self):
        if getattr(self, "h", None):
            for g in list(getattr(self.ctx, "_graphs", ())):
                if self in g.pops:
                    g.close()
            self.ctx.lib.spr_pop_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, sched, stream=None):
        self.ctx._check(self.ctx.lib.spr_run(self.h, sched.h, _stream_ptr(stream)))

    def sync(self):
        self.ctx._check(self.ctx.lib.spr_sync(self.h))

    def read(self, children=False):
        """Host copies: rho (P,N,N) complex64, supp (P,N,N) bool, err (P,) float64."""
        n, P = self.n, self.P
        rho = np.empty((P, n, n), dtype=np.complex64)
        supp = np.empty((P, n, n), dtype=np.uint8)
        err = np.empty(P, dtype=np.float64)
        flags = READ_CHILDREN if children else 0
        self.ctx._check(self.ctx.lib.spr_read(self.h, rho.ctypes.data, supp.ctypes.data,
                                              err.ctypes.data, flags))
        return rho, supp.astype(bool), err

    def monitors(self, max_n=4096):
        """Monitor records, oldest first, as dicts."""
        arr = (Monitor * max_n)()
        n = C.c_int32()
        self.ctx._check(self.ctx.lib.spr_read_monitor(self.h, arr, max_n, C.byref(n)))
        return [{k: getattr(arr[i], k) for k, _ in Monitor._fields_ if k != "pad"} for i in range(n.value)]

    def trace(self, max_rows=100000):
        """Fourier errors of the traced iterations of the last run: (rows, slots) float64."""
        rows, cols = C.c_int32(), C.c_int32()
        self.ctx._check(self.ctx.lib.spr_read_trace(self.h, None, 0, C.byref(rows), C.byref(cols)))
        k = min(rows.value, max_rows)
        out = np.empty((k, cols.value), dtype=np.float64)
        if k:
            self.ctx._check(self.ctx.lib.spr_read_trace(self.h, out.ctypes.data, k, C.byref(rows), C.byref(cols)))
        return out

    def init_spheres(self, sigma_init, n_init=5, diam=(0.2, 0.9), phase=(0.0, 0.0), gamma=1.0,
                     set_support=True):
        """The paper's sphere start for the parents, on the device (keyed by the population seed)."""
        prm = SphereParams(float(sigma_init), int(n_init), 1 if set_support else 0, float(diam[0]), float(diam[1]),
                           float(phase[0]), float(phase[1]), float(gamma))
        self.ctx._check(self.ctx.lib.spr_pop_init_spheres(self.h, C.byref(prm)))

    def average(self):
        """The last AVERAGE: rho (N,N) complex64, supp (N,N) bool, its fitness."""
        n = self.n
        rho = np.empty((n, n), dtype=np.complex64)
        supp = np.empty((n, n), dtype=np.uint8)
        err = np.empty(1, dtype=np.float64)
        self.ctx._check(self.ctx.lib.spr_read_average(self.h, rho.ctypes.data, supp.ctypes.data,
                                                      err.ctypes.data, 0))
        return rho, supp.astype(bool), float(err[0])

    def graph(self, sched):
        """Capture sched on this population into a replayable graph."""
        h = C.c_void_p()
        self.ctx._check(self.ctx.lib.spr_graph_create(self.h, sched.h, C.byref(h)))
        return Graph(self.ctx, h, [self])

    def read_member(self, member, children=False):
        """Host copies of one member: rho (N,N) complex64, supp (N,N) bool."""
        n = self.n
        rho = np.empty((n, n), dtype=np.complex64)
        supp = np.empty((n, n), dtype=np.uint8)
        flags = READ_CHILDREN if children else 0
        self.ctx._check(self.ctx.lib.spr_read_member(self.h, int(member), rho.ctypes.data, supp.ctypes.data,
                                                     flags))
        return rho, supp.astype(bool)

    def errors(self):
        """Fitness of the parents (P,) float64."""
        err = np.empty(self.P, dtype=np.float64)
        self.ctx._check(self.ctx.lib.spr_read(self.h, None, None, err.ctypes.data, 0))
        return err

    def read_into(self, rho=None, supp=None, err=None, children=False):
        """Read into caller tensors/arrays (all host or all device)."""
        ptrs = [_ptr(a) for a in (rho, supp, err)]
        devs = {d for (p, d) in ptrs if p is not None}
        if len(devs) > 1:
            raise ValueError("mix of host and device outputs")
        flags = (READ_CHILDREN if children else 0) | (DEVICE_PTRS if devs == {True} else 0)
        self.ctx._check(self.ctx.lib.spr_read(self.h, ptrs[0][0], ptrs[1][0], ptrs[2][0], flags))

    def write(self, rho=None, supp=None, err=None, children=False):
        ptrs = [_ptr(a) for a in (rho, supp, err)]
        devs = {d for (p, d) in ptrs if p is not None}
        if len(devs) > 1:
            raise ValueError("mix of host and device inputs")
        flags = (READ_CHILDREN if children else 0) | (DEVICE_PTRS if devs == {True} else 0)
        self.ctx._check(self.ctx.lib.spr_pop_write(self.h, ptrs[0][0], ptrs[1][0], ptrs[2][0], flags))

    def stats(self, max_n=4096):
        arr = (GenStats * max_n)()
        n = C.c_int32()
        self.ctx._check(self.ctx.lib.spr_read_stats(self.h, arr, max_n, C.byref(n)))
        return [arr[i] for i in range(n.value)]

    def timing(self, enable=True, kernels=None):
        """Enable per-launch event timing for the given kernel ids (default all)."""
        mask = 0
        if enable:
            mask = 0xF if kernels is None else sum(1 << k for k in kernels)
        self.ctx._check(self.ctx.lib.spr_timing_enable(self.h, mask))

    def timing_sample(self, every):
        """Time one launch in every `every` of each selected kernel (resets the totals)."""
        self.ctx._check(self.ctx.lib.spr_timing_sample(self.h, int(every)))

    def timing_read(self, kernel):
        """(launches, total event milliseconds) of one kernel since timing was enabled."""
        n = C.c_int64()
        ms = C.c_double()
        self.ctx._check(self.ctx.lib.spr_timing_read(self.h, int(kernel), C.byref(n), C.byref(ms)))
        return n.value, ms.value

    def xover(self):
        arr = (XoverInfo * self.P)()
        self.ctx._check(self.ctx.lib.spr_read_xover(self.h, arr, self.P))
        return [arr[i] for i in range(self.P)]


def op(kind, **kw):
    """Build an spr_op; unspecified fields are zero (chi defaults to 0.5)."""
    o = Op()
    o.kind = kind
    o.chi = 0.5
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Server:
    """Serving engine (continuous batching of streamed shots).

    ctx None selects the simulated executor (modelled time, no device work;
    manual stepping only).  submit() returns a ticket; poll(ticket) returns
    None until the shot is done, then a dict with the result and its
    arrival/admit/finish times (seconds on the server clock)."""

    def __init__(self, ctx, sched, P, hbm_budget, max_shots, manual=False, all_members=False,
                 max_inflight=0, max_queue=0, sim_bytes_per_s=0.0, sim_launch_s=0.0, shortest_first=False):
        self.lib = load()
        self.ctx = ctx
        self.P = int(P)
        self.all_members = bool(all_members)
        cfg = ServerCfg(int(hbm_budget), int(max_shots), self.P, sched.h.value if isinstance(sched.h, C.c_void_p)
                        else sched.h, (SERVER_MANUAL if manual else 0) | (SERVER_ALL_MEMBERS if all_members else 0)
                        | (SERVER_SHORTEST_FIRST if shortest_first else 0),
                        int(max_inflight), int(max_queue), float(sim_bytes_per_s), float(sim_launch_s))
        h = C.c_void_p()
        st = self.lib.spr_server_create(ctx.h if ctx else None, C.byref(cfg), C.byref(h))
        check(st, ctx.h if ctx else None)
        self.h = h
        self._n = {}
        if ctx is not None:
            ctx._servers.add(self)

    def _check(self, st):
        if st != SPR_OK:
            raw = self.lib.spr_server_last_error(self.h)
            raise SprError(st, raw.decode() if raw else "")

    def submit(self, amp, mask, supp0, rho0=None, seed=0, fft_order=False, arrival=None, fp16=False,
               bound_eta=0.0, bound_max_unknown=0.2, saturated=None, bound_max_saturated=0.05):
        """Queue one shot (host arrays); rho0 None = device random-phase start."""
        n = int(amp.shape[0])
        amp = np.ascontiguousarray(amp, dtype=np.float32)
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        supp0 = np.ascontiguousarray(supp0, dtype=np.uint8)
        flags = (LAYOUT_FFT if fft_order else 0) | (AMP_FP16 if fp16 else 0)
        if rho0 is None:
            flags |= INIT_RANDOM_PHASE
            rp = None
        else:
            rho0 = np.ascontiguousarray(rho0, dtype=np.complex64)
            rp = rho0.ctypes.data
        d = ShotDesc(n, amp.ctypes.data, mask.ctypes.data, supp0.ctypes.data, 1 if supp0.ndim == 3 else 0,
                     flags, rp, int(seed) & 0xFFFFFFFFFFFFFFFF, -1.0 if arrival is None else float(arrival),
                     float(bound_eta), float(bound_max_unknown), None, float(bound_max_saturated))
        if saturated is not None:
            saturated = np.ascontiguousarray(saturated, dtype=np.uint8)
            d.saturated = saturated.ctypes.data
        t = C.c_uint64()
        self._check(self.lib.spr_server_submit(self.h, C.byref(d), C.byref(t)))
        self._n[t.value] = n
        return t.value

    def poll(self, ticket, want_data=True):
        if ticket not in self._n:
            r = Result()
            self._check(self.lib.spr_server_poll(self.h, int(ticket), C.byref(r)))
        n = self._n[ticket]
        m = self.P if self.all_members else 1
        rho = np.empty((m, n, n), dtype=np.complex64) if want_data else None
        supp = np.empty((m, n, n), dtype=np.uint8) if want_data else None
        err = np.empty(self.P, dtype=np.float64)
        r = Result(rho.ctypes.data if want_data else None, supp.ctypes.data if want_data else None,
                   err.ctypes.data)
        st = self.lib.spr_server_poll(self.h, int(ticket), C.byref(r))
        if st == STATUS_NOT_READY:
            return None
        self._check(st)
        del self._n[ticket]
        return {"rho": rho, "supp": supp.astype(bool) if want_data else None, "err": err, "best": r.best,
                "members": r.members, "t_arrival": r.t_arrival, "t_admit": r.t_admit, "t_finish": r.t_finish,
                "status": r.status}

    def step(self):
        p = C.c_int64()
        self._check(self.lib.spr_server_step(self.h, C.byref(p)))
        return p.value

    def drain(self, timeout=-1.0):
        st = self.lib.spr_server_drain(self.h, float(timeout))
        if st == STATUS_NOT_READY:
            return False
        self._check(st)
        return True

    def stats(self):
        s = ServerStats()
        self._check(self.lib.spr_server_stats_get(self.h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "h", None):
            self.lib.spr_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """A schedule captured into a HIP graph; launch() replays it."""

    def __init__(self, ctx, h, pops):
        self.ctx = ctx
        self.h = h
        self.pops = list(pops)
        ctx._graphs.add(self)

    def launch(self, stream=None):
        self.ctx._check(self.ctx.lib.spr_graph_launch(self.h, _stream_ptr(stream)))

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.spr_graph_destroy(self.h)
            self.h = None
            self.pops = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
