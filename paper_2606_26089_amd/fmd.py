"""ctypes binding of libfmdet (include/fmd.h): argument marshalling only.

Every computation runs in the library's HIP kernels. Device arrays are torch tensors on
a ROCm device (torch provides device memory and the current HIP stream); host arrays are
NumPy arrays. Names follow the C ABI without the ``fmd_`` prefix.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfmdet.so")

OK, PENDING = 0, 1
E_INVALID, E_NOMEM, E_BUDGET, E_UNSUPPORTED, E_DEVICE, E_STATE = -1, -2, -3, -4, -5, -6
FP32, BF16, FP8 = 0, 1, 2
EULER, RK4, MIDPOINT = 0, 1, 2
(K_GEMM_QKV, K_GEMM_PROJ, K_GEMM_QC, K_GEMM_UP, K_GEMM_DOWN, K_FUSED_OQC, K_FUSED_MLP,
 K_ATTN_SELF, K_ATTN_CROSS, K_OTHER) = range(10)
FUSED_QKV, FUSED_OQC, FUSED_MLP, FUSED_EMBED, FUSED_ALL = 1, 2, 4, 8, 15
TUNE_ATTN_QUERY_TILE, TUNE_FUSED_QKV, TUNE_FUSED_OQC = 5, 6, 7
KERNEL_CLASSES = ("gemm_qkv", "gemm_proj", "gemm_qc", "gemm_up", "gemm_down", "fused_oqc",
                  "fused_mlp", "attn_self", "attn_cross", "other")

c_int32, c_int64, c_double, c_size_t, c_void_p = (ctypes.c_int32, ctypes.c_int64,
                                                    ctypes.c_double, ctypes.c_size_t,
                                                    ctypes.c_void_p)
P_int64 = ctypes.POINTER(ctypes.c_int64)


class ModelConfig(ctypes.Structure):
    _fields_ = [(n, c_int32) for n in ("d_model", "n_blocks", "n_heads", "mlp_ratio",
                                         "t_embed_dim", "f_truth", "f_reco", "n_max",
                                         "precision")]


class EventsIn(ctypes.Structure):
    _fields_ = [("n_events", c_int64), ("offsets", P_int64), ("feat", c_void_p),
                ("on_device", c_int32)]


class EventsOut(ctypes.Structure):
    _fields_ = [("feat", c_void_p), ("on_device", c_int32)]


class Schedule(ctypes.Structure):
    _fields_ = [("scheme", c_int32), ("n_steps", c_int32), ("t0", c_double), ("t1", c_double)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", c_size_t), ("max_tokens_per_iter", c_int64),
                ("max_requests", c_int32)]


class RequestStats(ctypes.Structure):
    _fields_ = [("t_submit_ns", ctypes.c_uint64), ("t_admit_ns", ctypes.c_uint64),
                ("t_done_ns", ctypes.c_uint64)]


class ServerInfo(ctypes.Structure):
    _fields_ = [(n, c_int64) for n in ("pool_tokens", "bytes_per_token", "queued_requests",
                                        "resident_requests", "resident_tokens", "iterations",
                                        "rows_processed", "busy_ns", "rows_live")]


class MultiplicityLaw(ctypes.Structure):
    _fields_ = [("loss_prob", ctypes.c_double), ("fake_prob", ctypes.c_double),
                ("fake_trials", c_int32)]


class FmdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"fmd status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libfmdet.so; raise if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2606_26089_amd.build` (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "fmd_last_error": (ctypes.c_char_p, []),
        "fmd_param_count": (c_size_t, [ctypes.POINTER(ModelConfig)]),
        "fmd_model_create": (c_int32, [ctypes.POINTER(ModelConfig), c_void_p, c_size_t,
                                       ctypes.POINTER(c_void_p)]),
        "fmd_model_destroy": (c_int32, [c_void_p]),
        "fmd_linear_field_create": (c_int32, [c_double, c_double, ctypes.POINTER(c_void_p)]),
        "fmd_simulate": (c_int32, [c_void_p, ctypes.POINTER(EventsIn), ctypes.c_uint64,
                                   ctypes.POINTER(Schedule), ctypes.POINTER(EventsOut), c_void_p]),
        "fmd_simulate_reco": (c_int32, [c_void_p, ctypes.POINTER(EventsIn), P_int64,
                                        ctypes.c_uint64, ctypes.POINTER(Schedule),
                                        ctypes.POINTER(EventsOut), c_void_p]),
        "fmd_simulate_from_state": (c_int32, [c_void_p, ctypes.POINTER(EventsIn), c_void_p,
                                              ctypes.POINTER(Schedule), ctypes.POINTER(EventsOut),
                                              c_void_p]),
        "fmd_velocity": (c_int32, [c_void_p, ctypes.POINTER(EventsIn), c_void_p, c_void_p,
                                   c_void_p, c_void_p]),
        "fmd_noise": (c_int32, [ctypes.c_uint64, P_int64, c_int64, c_int32, c_void_p, c_void_p]),
        "fmd_event_observables": (c_int32, [ctypes.POINTER(EventsIn), c_void_p, c_void_p, c_void_p,
                                            c_void_p]),
        "fmd_truth_select": (c_int32, [ctypes.POINTER(EventsIn), ctypes.c_double, c_int32, P_int64,
                                       c_void_p, c_void_p]),
        "fmd_reco_multiplicity": (c_int32, [P_int64, c_int64, ctypes.c_uint64,
                                            ctypes.POINTER(MultiplicityLaw), c_int32, P_int64,
                                            c_void_p]),
        "fmd_truth_select_noalloc": (c_int32, [ctypes.POINTER(EventsIn), ctypes.c_double, c_int32,
                                               P_int64, c_void_p, c_void_p]),
        "fmd_debug_philox": (c_int32, [ctypes.c_uint64, ctypes.c_uint64, c_void_p, c_int64,
                                       c_void_p, c_void_p]),
        "fmd_pack_padded": (c_int32, [c_void_p, c_void_p, c_int64, c_int32, c_int32, c_void_p,
                                      c_void_p, c_void_p]),
        "fmd_timing_enable": (c_int32, [c_void_p, c_int32]),
        "fmd_timing_read": (c_int32, [c_void_p, c_int32, ctypes.POINTER(c_double),
                                      ctypes.POINTER(c_int64), ctypes.POINTER(c_double),
                                      ctypes.POINTER(c_double)]),
        "fmd_kernel_name": (ctypes.c_char_p, [c_void_p, c_int32]),
        "fmd_autotune_enable": (c_int32, [c_void_p, c_int32]),
        "fmd_graphs_enable": (c_int32, [c_void_p, c_int32]),
        "fmd_fused_enable": (c_int32, [c_void_p, c_int32]),
        "fmd_tuning_table": (c_int32, [c_void_p, ctypes.c_char_p, c_size_t, ctypes.POINTER(c_size_t)]),
        "fmd_tuning_set": (c_int32, [c_void_p, c_int32, c_int32, c_int32]),
        "fmd_server_create": (c_int32, [c_void_p, ctypes.POINTER(ServerConfig), ctypes.POINTER(c_void_p)]),
        "fmd_server_submit": (c_int32, [c_void_p, ctypes.POINTER(EventsIn), ctypes.c_uint64,
                                        ctypes.POINTER(Schedule), ctypes.POINTER(ctypes.c_uint64)]),
        "fmd_server_submit_reco": (c_int32, [c_void_p, ctypes.POINTER(EventsIn), P_int64,
                                             ctypes.c_uint64, ctypes.POINTER(Schedule),
                                             ctypes.POINTER(ctypes.c_uint64)]),
        "fmd_server_poll": (c_int32, [c_void_p, ctypes.c_uint64, c_void_p, ctypes.POINTER(RequestStats)]),
        "fmd_server_wait": (c_int32, [c_void_p, ctypes.c_uint64, c_void_p, ctypes.POINTER(RequestStats)]),
        "fmd_server_get_info": (c_int32, [c_void_p, ctypes.POINTER(ServerInfo)]),
        "fmd_server_destroy": (c_int32, [c_void_p]),
        "fmd_debug_gemm": (c_int32, [c_int32, c_int64, c_int32, c_int32, c_void_p, c_void_p,
                                     c_void_p, c_int32, c_void_p, c_void_p, c_int32, c_void_p,
                                     c_int32, c_void_p]),
        "fmd_debug_attention": (c_int32, [c_int32, c_int64, P_int64, P_int64, c_int32, c_int32,
                                          c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(status):
    if status != OK and status != PENDING:
        raise FmdError(status, lib().fmd_last_error().decode())
    return status


# ---------------------------------------------------------------------------------------
# marshalling helpers

def _is_torch(a):
    return type(a).__module__.startswith("torch")


def _stream(stream):
    if stream is not None:
        return c_void_p(int(stream))
    import torch
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(a):
    """(pointer, on_device) of a float32 C-contiguous host array or device tensor."""
    if a is None:
        return None, 0
    if _is_torch(a):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return c_void_p(a.data_ptr()), int(a.is_cuda)
    if not (isinstance(a, np.ndarray) and a.flags.c_contiguous):
        raise ValueError("host arrays must be C-contiguous NumPy arrays")
    return c_void_p(a.ctypes.data), 0


def _offsets(offsets):
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    return off, off.ctypes.data_as(P_int64)


def _events(offsets, feat):
    off, p = _offsets(offsets)
    fp, dev = _ptr(feat)
    return EventsIn(len(off) - 1, p, fp, dev), off


def model_config(cfg) -> ModelConfig:
    """Accepts any object with the fields of fmd_model_config (or a dict)."""
    get = cfg.get if isinstance(cfg, dict) else (lambda k: getattr(cfg, k))
    return ModelConfig(*[int(get(n)) for n, _ in ModelConfig._fields_])


def schedule(s) -> Schedule:
    if isinstance(s, Schedule):
        return s
    get = s.get if isinstance(s, dict) else (lambda k: getattr(s, k))
    return Schedule(int(get("scheme")), int(get("n_steps")), float(get("t0")), float(get("t1")))


def param_count(cfg) -> int:
    c = model_config(cfg)
    return int(lib().fmd_param_count(ctypes.byref(c)))


def _like_out(feat, rows, cols):
    if _is_torch(feat):
        import torch
        return torch.empty((rows, cols), dtype=torch.float32, device=feat.device)
    return np.empty((rows, cols), dtype=np.float32)


# ---------------------------------------------------------------------------------------
# model

class Model:
    """A velocity network (or the analytic linear test field) on the current HIP device."""

    def __init__(self, cfg=None, params=None, *, _handle=None):
        L = lib()
        if _handle is not None:
            self._h = _handle
            self.cfg = None
            return
        c = model_config(cfg)
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        h = c_void_p()
        _check(L.fmd_model_create(ctypes.byref(c), c_void_p(p.ctypes.data), p.size, ctypes.byref(h)))
        self._h = h
        self.cfg = cfg

    @classmethod
    def linear_field(cls, alpha, beta):
        h = c_void_p()
        _check(lib().fmd_linear_field_create(float(alpha), float(beta), ctypes.byref(h)))
        return cls(_handle=h)

    def close(self):
        if getattr(self, "_h", None):
            lib().fmd_model_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def simulate(self, offsets, feat, seed, sched, out=None, stream=None, reco_offsets=None):
        """Reco state at t1 [T, 9]; with reco_offsets ([E + 1] host ints) the events get that
        many reco slots each (fmd_simulate_reco) and the result is [reco_offsets[-1], 9]."""
        ev, off = _events(offsets, feat)
        roff = None
        if reco_offsets is not None:
            roff = np.ascontiguousarray(np.asarray(reco_offsets, dtype=np.int64))
            if len(roff) != len(off):
                raise ValueError("reco_offsets needs one entry per event plus one")
        rows = int(off[-1]) if roff is None else int(roff[-1])
        if out is None:
            out = _like_out(feat, rows, 9)
        op, odev = _ptr(out)
        o = EventsOut(op, odev)
        s = schedule(sched)
        st = _stream(stream) if ev.on_device or odev else None
        if roff is None:
            _check(lib().fmd_simulate(self._h, ctypes.byref(ev), ctypes.c_uint64(seed),
                                      ctypes.byref(s), ctypes.byref(o), st))
        else:
            _check(lib().fmd_simulate_reco(self._h, ctypes.byref(ev), roff.ctypes.data_as(P_int64),
                                           ctypes.c_uint64(seed), ctypes.byref(s),
                                           ctypes.byref(o), st))
        return out

    def simulate_from_state(self, offsets, feat, x0, sched, out=None, stream=None):
        ev, off = _events(offsets, feat)
        if out is None:
            out = _like_out(feat, int(off[-1]), 9)
        op, odev = _ptr(out)
        xp, _ = _ptr(x0)
        o = EventsOut(op, odev)
        s = schedule(sched)
        _check(lib().fmd_simulate_from_state(self._h, ctypes.byref(ev), xp, ctypes.byref(s),
                                             ctypes.byref(o),
                                             _stream(stream) if ev.on_device or odev else None))
        return out

    def velocity(self, offsets, feat, x, t_per_event, out=None, stream=None):
        ev, off = _events(offsets, feat)
        if out is None:
            out = _like_out(feat, int(off[-1]), 9)
        xp, _ = _ptr(x)
        tp, _ = _ptr(t_per_event)
        vp, _ = _ptr(out)
        _check(lib().fmd_velocity(self._h, ctypes.byref(ev), xp, tp, vp,
                                  _stream(stream) if ev.on_device else None))
        return out

    def timing_enable(self, on=True):
        _check(lib().fmd_timing_enable(self._h, int(bool(on))))

    def timing_read(self, cls):
        """(device ms, launches, algorithmic FLOPs, algorithmic HBM bytes) of one class."""
        ms, n, work, nb = c_double(), c_int64(), c_double(), c_double()
        _check(lib().fmd_timing_read(self._h, int(cls), ctypes.byref(ms), ctypes.byref(n),
                                     ctypes.byref(work), ctypes.byref(nb)))
        return ms.value, n.value, work.value, nb.value

    def graphs_enable(self, on=True):
        _check(lib().fmd_graphs_enable(self._h, int(bool(on))))

    def fused_enable(self, on=True):
        """True: every fused block kernel; False: none; an int: FUSED_* bit mask."""
        mask = FUSED_ALL if on is True else 0 if on is False else int(on)
        _check(lib().fmd_fused_enable(self._h, mask))

    def autotune_enable(self, on=True):
        _check(lib().fmd_autotune_enable(self._h, int(bool(on))))

    def tuning_table(self):
        import json
        need = c_size_t()
        _check(lib().fmd_tuning_table(self._h, None, 0, ctypes.byref(need)))
        buf = ctypes.create_string_buffer(need.value)
        _check(lib().fmd_tuning_table(self._h, buf, need.value, None))
        return json.loads(buf.value.decode())

    def tuning_set(self, site, tokens_log2, candidate):
        """Fixes the autotuner's choice for a fused-path site (TUNE_ATTN_QUERY_TILE,
        TUNE_FUSED_QKV, TUNE_FUSED_OQC) and a log2 token bucket: candidate 0 (64) or 1 (128);
        the attention site also has 2 (192 queries per work item)."""
        _check(lib().fmd_tuning_set(self._h, int(site), int(tokens_log2), int(candidate)))

    def kernel_name(self, cls):
        return lib().fmd_kernel_name(self._h, int(cls)).decode()


class Server:
    """Continuous-batching server over a Model (see fmd_server_* in include/fmd.h)."""

    def __init__(self, model, hbm_budget_bytes, max_tokens_per_iter=0, max_requests=0):
        cfg = ServerConfig(int(hbm_budget_bytes), int(max_tokens_per_iter), int(max_requests))
        h = c_void_p()
        _check(lib().fmd_server_create(model._h, ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self.model = model
        self._sizes = {}

    def submit(self, offsets, feat, seed, sched, reco_offsets=None):
        """Queues a request; with reco_offsets ([E + 1] ints) its events get that many reco
        slots each (fmd_server_submit_reco)."""
        feat = np.ascontiguousarray(np.asarray(feat, dtype=np.float32))
        ev, off = _events(offsets, feat)
        s = schedule(sched)
        rid = ctypes.c_uint64()
        # the library copies the request before returning
        if reco_offsets is None:
            rows = int(off[-1])
            _check(lib().fmd_server_submit(self._h, ctypes.byref(ev), ctypes.c_uint64(seed),
                                           ctypes.byref(s), ctypes.byref(rid)))
        else:
            roff = np.ascontiguousarray(np.asarray(reco_offsets, dtype=np.int64))
            if len(roff) != len(off):
                raise ValueError("reco_offsets needs one entry per event plus one")
            rows = int(roff[-1])
            _check(lib().fmd_server_submit_reco(self._h, ctypes.byref(ev),
                                                roff.ctypes.data_as(P_int64),
                                                ctypes.c_uint64(seed), ctypes.byref(s),
                                                ctypes.byref(rid)))
        self._sizes[rid.value] = rows
        return rid.value

    def _collect(self, fn, rid):
        out = np.empty((self._sizes[rid], 9), dtype=np.float32)
        st = RequestStats()
        status = fn(self._h, ctypes.c_uint64(rid), c_void_p(out.ctypes.data), ctypes.byref(st))
        if status == PENDING:
            return None
        self._sizes.pop(rid, None)
        _check(status)
        return out, {"t_submit_ns": st.t_submit_ns, "t_admit_ns": st.t_admit_ns,
                     "t_done_ns": st.t_done_ns}

    def poll(self, rid):
        """(reco, stats) once finished, else None."""
        return self._collect(lib().fmd_server_poll, rid)

    def wait(self, rid):
        return self._collect(lib().fmd_server_wait, rid)

    def info(self):
        i = ServerInfo()
        _check(lib().fmd_server_get_info(self._h, ctypes.byref(i)))
        return {n: getattr(i, n) for n, _ in ServerInfo._fields_}

    def close(self):
        if getattr(self, "_h", None):
            lib().fmd_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def linear_field(alpha, beta):
    return Model.linear_field(alpha, beta)


def noise(seed, offsets, n_feat, out, stream=None):
    """x0 noise into a device tensor out [offsets[-1], n_feat]."""
    off, p = _offsets(offsets)
    op, dev = _ptr(out)
    if not dev:
        raise ValueError("noise writes device memory: pass a device tensor")
    _check(lib().fmd_noise(ctypes.c_uint64(seed), p, len(off) - 1, int(n_feat), op, _stream(stream)))
    return out


def event_observables(offsets, feat, stream=None):
    """(ht [E], met [E], iso [T]) of reconstructed events feat [T, 9] (Sec. 2.4): H_T, MET and
    lepton isolation (NaN for other classes). Outputs live where feat lives (NumPy on the
    host, torch tensors on its device)."""
    ev, off = _events(offsets, feat)
    E, T = len(off) - 1, int(off[-1])
    if _is_torch(feat):
        import torch
        ht = torch.empty(E, dtype=torch.float32, device=feat.device)
        met = torch.empty(E, dtype=torch.float32, device=feat.device)
        iso = torch.empty(T, dtype=torch.float32, device=feat.device)
        ptrs = [c_void_p(t.data_ptr()) for t in (ht, met, iso)]
    else:
        ht, met, iso = np.empty(E, np.float32), np.empty(E, np.float32), np.empty(T, np.float32)
        ptrs = [c_void_p(a.ctypes.data) for a in (ht, met, iso)]
    _check(lib().fmd_event_observables(ctypes.byref(ev), *ptrs, _stream(stream)))
    return ht, met, iso


def truth_select(offsets, feat, pt_cut_gev, max_particles, stream=None):
    """(offsets_out [E+1] int64 NumPy, feat_out [offsets_out[-1], 9]) after the model's truth
    selection: pT > pt_cut_gev, at most max_particles per event (the hardest), input order.
    feat_out lives where feat lives."""
    ev, off = _events(offsets, feat)
    T = int(off[-1])
    out_off = np.zeros(len(off), dtype=np.int64)
    if _is_torch(feat):
        import torch
        out = torch.empty((T, 9), dtype=torch.float32, device=feat.device)
        op = c_void_p(out.data_ptr())
    else:
        out = np.empty((T, 9), dtype=np.float32)
        op = c_void_p(out.ctypes.data)
    _check(lib().fmd_truth_select(ctypes.byref(ev), float(pt_cut_gev), int(max_particles),
                                  out_off.ctypes.data_as(P_int64), op, _stream(stream)))
    return out_off, out[: int(out_off[-1])]


def reco_multiplicity(offsets, seed, loss_prob, fake_prob, fake_trials, n_max, stream=None):
    """Reco offsets [E+1] int64 (NumPy) drawn on the device under the stand-in multiplicity
    law (truth particles missed with probability loss_prob, Binomial(fake_trials, fake_prob)
    extra slots, at most n_max per event), to pass as reco_offsets to Model.simulate."""
    off, p = _offsets(offsets)
    out = np.zeros(len(off), dtype=np.int64)
    law = MultiplicityLaw(float(loss_prob), float(fake_prob), int(fake_trials))
    _check(lib().fmd_reco_multiplicity(p, len(off) - 1, ctypes.c_uint64(seed & (2**64 - 1)),
                                       ctypes.byref(law), int(n_max), out.ctypes.data_as(P_int64),
                                       _stream(stream)))
    return out


def truth_select_noalloc(offsets, feat, pt_cut_gev, max_particles, out, stream=None):
    """As truth_select for device data, through the entry point that allocates no device
    memory: feat [T, 9] and out (capacity T rows) are caller-owned device tensors. Returns
    (offsets_out [E+1] int64 NumPy, out[:offsets_out[-1]])."""
    ev, off = _events(offsets, feat)
    out_off = np.zeros(len(off), dtype=np.int64)
    _check(lib().fmd_truth_select_noalloc(ctypes.byref(ev), float(pt_cut_gev), int(max_particles),
                                          out_off.ctypes.data_as(P_int64), c_void_p(out.data_ptr()),
                                          _stream(stream)))
    return out_off, out[: int(out_off[-1])]


def pack_padded(padded, lengths, offsets_out, feat_out, stream=None):
    """Device tensors: padded [E, n_max, f] f32, lengths [E] int32 -> offsets_out [E+1] int64,
    feat_out [E * n_max, f] (first offsets_out[-1] rows valid)."""
    E, n_max, f = padded.shape
    _check(lib().fmd_pack_padded(c_void_p(padded.data_ptr()), c_void_p(lengths.data_ptr()), E,
                                 n_max, f, c_void_p(offsets_out.data_ptr()),
                                 c_void_p(feat_out.data_ptr()), _stream(stream)))
    return offsets_out, feat_out


def debug_philox(key0, key1, counters, out=None, stream=None):
    """Device uint64 tensors (torch.int64 storage): counters [n, 4] -> out [n, 4]."""
    import torch
    if out is None:
        out = torch.empty_like(counters)
    _check(lib().fmd_debug_philox(ctypes.c_uint64(key0), ctypes.c_uint64(key1),
                                  c_void_p(counters.data_ptr()), counters.shape[0],
                                  c_void_p(out.data_ptr()), _stream(stream)))
    return out


def debug_gemm(precision, A, W, bias=None, ln=None, epi=0, C=None, tile=-1, stream=None):
    """Device float32 tensors: A [M, K], W [K, N]; ln = (g, s) or None; epi 0/1/2;
    tile = candidate tiling (-1 default)."""
    import torch
    M, K = A.shape
    N = W.shape[1]
    if C is None:
        C = torch.zeros((M, N), dtype=torch.float32, device=A.device)
    g, s = ln if ln is not None else (None, None)
    P = lambda t: c_void_p(t.data_ptr()) if t is not None else None  # noqa: E731
    _check(lib().fmd_debug_gemm(int(precision), M, N, K, P(A), P(W), P(bias), int(ln is not None),
                                P(g), P(s), int(epi), P(C), int(tile), _stream(stream)))
    return C


def debug_attention(precision, q_offsets, kv_offsets, n_heads, dh, Q, K, V, O=None, stream=None):
    import torch
    qo, qp = _offsets(q_offsets)
    ko, kp = _offsets(kv_offsets)
    if O is None:
        O = torch.zeros_like(Q)
    P = lambda t: c_void_p(t.data_ptr())  # noqa: E731
    _check(lib().fmd_debug_attention(int(precision), len(qo) - 1, qp, kp, int(n_heads), int(dh),
                                     P(Q), P(K), P(V), P(O), _stream(stream)))
    return O
