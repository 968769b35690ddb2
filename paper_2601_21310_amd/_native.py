"""ctypes binding of libdnqs.so (the C ABI in include/dnqs.h).

Argument marshalling only: every step of the hot path runs in the library's HIP
kernels.  PyTorch provides device memory and the stream.  There is no fallback: if
the library is not built, or no gfx950 GPU is present, calls raise.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdnqs.so")

MAX_LAYERS = 8
FP32, MIXED, SPLIT_BF16 = 0, 1, 2
VALIDATE = 1
EMIT_P = 2
EMIT_HPS = 4
FULL_OUTPUT = 1
ASYM = 2
ASYM_ESTIMATOR = 4
RECOMPUTE = 8

STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ECAPACITY", -5: "ESTATE", -6: "EDOMAIN"}


class DnqsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"dnqs {STATUS.get(status, status)}: {msg}")
        self.status = status


class Net(C.Structure):
    _fields_ = [("n_layers", C.c_int), ("width", C.c_int * (MAX_LAYERS + 1))]

    @classmethod
    def from_widths(cls, widths):
        w = list(widths)
        if not 3 <= len(w) <= MAX_LAYERS + 1:
            raise ValueError("need between 3 and 9 widths (2 to 8 layers)")
        net = cls()
        net.n_layers = len(w) - 1
        for i, v in enumerate(w):
            net.width[i] = int(v)
        return net


class Problem(C.Structure):
    _fields_ = [("slot", C.c_int), ("conn", C.c_void_p), ("theta", C.c_void_p), ("grad", C.c_void_p),
                ("energy", C.c_void_p), ("stats", C.c_void_p)]


class AdamwCfg(C.Structure):
    _fields_ = [("lr_max", C.c_float), ("lr_min", C.c_float), ("decay_steps", C.c_int), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float), ("weight_decay", C.c_float)]


class PT2Opts(C.Structure):
    _fields_ = [("sample_mask", C.c_uint64), ("export_cap", C.c_int64), ("export_keys", C.c_void_p),
                ("export_w", C.c_void_p), ("export_haa", C.c_void_p), ("export_count", C.c_void_p),
                ("max_pair_bytes", C.c_int64), ("eps_hb", C.c_double)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


# connection sets, graphs and contexts still open when the interpreter exits are freed
# (in that order) while torch, whose caching allocator takes back their device memory,
# is still alive
_open_objects = weakref.WeakSet()
_open_contexts = weakref.WeakSet()


@atexit.register
def _close_open_contexts():
    for o in list(_open_objects):
        try:
            o.free()
        except Exception:
            pass
    for c in list(_open_contexts):
        try:
            c.close()
        except Exception:
            pass


class TorchAllocator:
    """Device memory for the library from torch's caching allocator, on the context's
    stream (torch stays the only owner of device memory).  Counts calls and live bytes."""

    def __init__(self, device: int, stream: int):
        self.device = device
        self.stream = stream
        self._delete = torch.cuda.caching_allocator_delete
        self.n_alloc = 0
        self.n_release = 0
        self.live = {}

    def alloc(self, nbytes: int):
        try:
            p = torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
        except torch.cuda.OutOfMemoryError:
            return None
        self.n_alloc += 1
        self.live[p] = int(nbytes)
        return p

    def release(self, p: int):
        self.n_release += 1
        self.live.pop(p, None)
        self._delete(p)

    @property
    def live_bytes(self):
        return sum(self.live.values())


_lib = None


def lib():
    """Load libdnqs.so; raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                              "python paper_2601_21310_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32, u64, dbl = C.c_void_p, C.c_int64, C.c_int, C.c_uint64, C.c_double
        L.dnqs_create.argtypes = [C.POINTER(vp), i32, vp, ALLOC_FN, RELEASE_FN, vp]
        L.dnqs_destroy.argtypes = [vp]
        L.dnqs_destroy.restype = None
        L.dnqs_set_stream.argtypes = [vp, vp]
        L.dnqs_last_error.argtypes = [vp]
        L.dnqs_last_error.restype = C.c_char_p
        L.dnqs_param_count.argtypes = [C.POINTER(Net), i32, i32, i32]
        L.dnqs_param_count.restype = i64
        L.dnqs_set_integrals.argtypes = [vp, i32, i32, i32, i32, vp, vp, dbl]
        L.dnqs_build_connections.argtypes = [vp, i32, vp, i64, C.c_uint, C.POINTER(vp)]
        L.dnqs_conn_info.argtypes = [vp, C.POINTER(i64), C.POINTER(i64)]
        L.dnqs_conn_output_plan.argtypes = [vp, C.POINTER(i32), C.POINTER(i64)]
        L.dnqs_conn_p_info.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(u64)]
        L.dnqs_build_target.argtypes = [vp, i32, vp, vp, i64, C.c_uint, C.POINTER(vp)]
        L.dnqs_conn_export_p.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.dnqs_conn_export.argtypes = [vp, vp, vp, vp, vp, vp]
        L.dnqs_conn_free.argtypes = [vp]
        L.dnqs_conn_free.restype = None
        L.dnqs_amplitudes.argtypes = [vp, i32, C.POINTER(Net), vp, vp, i64, i32, vp, vp]
        L.dnqs_energy_and_grad.argtypes = [vp, i32, C.POINTER(Net), vp, vp, i32, C.c_uint, vp, vp, vp, vp, vp, vp]
        L.dnqs_pt2.argtypes = [vp, i32, vp, vp, vp, vp, C.POINTER(PT2Opts), vp, vp]
        L.dnqs_lanczos.argtypes = [vp, vp, i32, dbl, vp, vp, vp, C.POINTER(i32), C.POINTER(dbl)]
        L.dnqs_heatbath_candidates.argtypes = [vp, i32, vp, vp, vp, dbl, i64, vp, C.POINTER(i64)]
        L.dnqs_select_topk.argtypes = [vp, i32, vp, vp, vp, i64, i64, vp, C.POINTER(i64)]
        L.dnqs_energy_and_grad_batched.argtypes = [vp, C.POINTER(Net), i32, C.POINTER(Problem), i32, C.c_uint]
        L.dnqs_adamw_batched.argtypes = [vp, C.POINTER(Net), i32, C.POINTER(Problem), vp, vp, C.POINTER(AdamwCfg), vp]
        L.dnqs_capture_begin.argtypes = [vp]
        L.dnqs_capture_end.argtypes = [vp, C.POINTER(vp)]
        L.dnqs_graph_launch.argtypes = [vp, vp]
        L.dnqs_graph_free.argtypes = [vp]
        L.dnqs_graph_free.restype = None
        L.dnqs_timing_enable.argtypes = [vp, i32]
        L.dnqs_timing_reset.argtypes = [vp]
        L.dnqs_timing_get.argtypes = [vp, C.c_char_p, C.POINTER(dbl), C.POINTER(i64)]
        L.dnqs_autotune.argtypes = [vp, i32]
        L.dnqs_tune_export.argtypes = [vp, C.c_char_p, i64]
        L.dnqs_tune_export.restype = i64
        L.dnqs_tune_import.argtypes = [vp, C.c_char_p]
        for fn in ("dnqs_create", "dnqs_set_stream", "dnqs_set_integrals", "dnqs_build_connections",
                   "dnqs_conn_info", "dnqs_conn_output_plan", "dnqs_build_target", "dnqs_conn_export", "dnqs_conn_p_info", "dnqs_conn_export_p", "dnqs_amplitudes", "dnqs_energy_and_grad", "dnqs_pt2", "dnqs_lanczos",
                   "dnqs_heatbath_candidates", "dnqs_select_topk",
                   "dnqs_energy_and_grad_batched", "dnqs_adamw_batched", "dnqs_capture_begin", "dnqs_capture_end",
                   "dnqs_graph_launch", "dnqs_timing_enable", "dnqs_timing_reset", "dnqs_timing_get",
                   "dnqs_autotune", "dnqs_tune_import"):
            getattr(L, fn).restype = C.c_int
        _lib = L
    return _lib


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _dev_tensor(t, dtype, name, device):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda" or t.device.index != device:
        raise ValueError(f"{name} must live on cuda:{device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


class Connections:
    """H_SS of a variational set (library-owned device memory)."""

    def __init__(self, ctx, handle, slot, dets):
        self._ctx = ctx
        self.handle = handle
        _open_objects.add(self)
        self.slot = slot
        self.dets = dets
        n, nnz = C.c_int64(), C.c_int64()
        lib().dnqs_conn_info(handle, C.byref(n), C.byref(nnz))
        self.n, self.nnz = n.value, nnz.value

    def output_plan(self):
        """(dense orbitals or -1 when the full-width output layer is used, sparse rows)."""
        nd, ne = C.c_int32(), C.c_int64()
        lib().dnqs_conn_output_plan(self.handle, C.byref(nd), C.byref(ne))
        return nd.value, ne.value

    def export(self):
        """(row_ptr int64, col int32, val float32, diag float64) as CUDA tensors."""
        dev = self._ctx.device
        row_ptr = torch.empty(self.n + 1, dtype=torch.int64, device=f"cuda:{dev}")
        col = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=f"cuda:{dev}")
        val = torch.empty(max(self.nnz, 1), dtype=torch.float32, device=f"cuda:{dev}")
        diag = torch.empty(self.n, dtype=torch.float64, device=f"cuda:{dev}")
        self._ctx._check(lib().dnqs_conn_export(self._ctx.handle, self.handle, _ptr(row_ptr), _ptr(col),
                                                 _ptr(val), _ptr(diag)))
        torch.cuda.current_stream(dev).synchronize()
        return row_ptr, col[: self.nnz], val[: self.nnz], diag

    def p_info(self):
        """(|P|, nnz(H_PS) or -1, (fingerprint sum, fingerprint xor)) of a set built with emit_p."""
        np_, nnz = C.c_int64(), C.c_int64()
        fp = (C.c_uint64 * 2)()
        self._ctx._check(lib().dnqs_conn_p_info(self.handle, C.byref(np_), C.byref(nnz), fp))
        return np_.value, nnz.value, (int(fp[0]), int(fp[1]))

    def export_p(self):
        """(P int64[|P|,2], H_aa float64, and when built H_PS row_ptr int64, col int32, val float32)."""
        dev = self._ctx.device
        n_p, nnz, _ = self.p_info()
        pd = torch.empty((max(n_p, 1), 2), dtype=torch.int64, device=f"cuda:{dev}")
        pdiag = torch.empty(max(n_p, 1), dtype=torch.float64, device=f"cuda:{dev}")
        rp = col = val = None
        if nnz >= 0:
            rp = torch.empty(n_p + 1, dtype=torch.int64, device=f"cuda:{dev}")
            col = torch.empty(max(nnz, 1), dtype=torch.int32, device=f"cuda:{dev}")
            val = torch.empty(max(nnz, 1), dtype=torch.float32, device=f"cuda:{dev}")
        self._ctx._check(lib().dnqs_conn_export_p(self._ctx.handle, self.handle, _ptr(pd), _ptr(pdiag), _ptr(rp),
                                                   _ptr(col), _ptr(val)))
        torch.cuda.current_stream(dev).synchronize()
        res = {"p": pd[:n_p], "diag": pdiag[:n_p]}
        if nnz >= 0:
            res.update(row_ptr=rp, col=col[:nnz], val=val[:nnz])
        return res

    def free(self):
        if self.handle:
            lib().dnqs_conn_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Context:
    """One library context on one GPU, enqueuing on torch's current stream.

    allocator: "torch" (default: torch's caching allocator, a TorchAllocator), None (the
    library's own hipMalloc / hipFree) or an object with alloc(nbytes) -> int or None and
    release(ptr)."""

    def __init__(self, device: int = 0, allocator="torch"):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the dnqs library runs only on gfx950 GPUs")
        self.device = device
        h = C.c_void_p()
        stream = torch.cuda.current_stream(device).cuda_stream
        if allocator == "torch":
            allocator = TorchAllocator(device, stream)
        self.allocator = allocator
        if allocator is None:
            self._cb = (ALLOC_FN(), RELEASE_FN())
        else:
            def _alloc(nbytes, user, _a=allocator):
                try:
                    return _a.alloc(nbytes)
                except Exception:
                    return None

            def _release(p, user, _a=allocator):
                _a.release(p)

            self._cb = (ALLOC_FN(_alloc), RELEASE_FN(_release))
        st = lib().dnqs_create(C.byref(h), device, C.c_void_p(stream), self._cb[0], self._cb[1], None)
        if st != 0:
            raise DnqsError(st, lib().dnqs_last_error(None).decode())
        self.handle = h
        self.stream = stream
        self._slots = {}
        _open_contexts.add(self)

    def _check(self, st):
        if st != 0:
            raise DnqsError(st, lib().dnqs_last_error(self.handle).decode())

    def sync_stream(self):
        """Point the context at torch's current stream."""
        stream = torch.cuda.current_stream(self.device).cuda_stream
        self._check(lib().dnqs_set_stream(self.handle, C.c_void_p(stream)))
        self.stream = stream
        if isinstance(self.allocator, TorchAllocator):
            self.allocator.stream = stream

    def close(self):
        if getattr(self, "handle", None):
            lib().dnqs_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------- calls
    def set_integrals(self, h, eri, e_core, n_alpha, n_beta, slot=0):
        h = np.ascontiguousarray(h, dtype=np.float64)
        eri = np.ascontiguousarray(eri, dtype=np.float64)
        M = h.shape[0]
        if h.shape != (M, M) or eri.shape != (M, M, M, M):
            raise ValueError("h must be [M,M] and eri [M,M,M,M]")
        self._check(lib().dnqs_set_integrals(self.handle, slot, M, n_alpha, n_beta, h.ctypes.data_as(C.c_void_p),
                                              eri.ctypes.data_as(C.c_void_p), float(e_core)))
        self._slots[slot] = (M, n_alpha, n_beta)

    def shape(self, slot=0):
        return self._slots[slot]

    def build_connections(self, dets, slot=0, validate=True, emit_p=False, emit_hps=False) -> Connections:
        dets = _dev_tensor(dets, torch.int64, "dets", self.device)
        n = dets.shape[0]
        h = C.c_void_p()
        flags = (VALIDATE if validate else 0) | (EMIT_P if emit_p else 0) | (EMIT_HPS if emit_hps else 0)
        self._check(lib().dnqs_build_connections(self.handle, slot, _ptr(dets), n, flags, C.byref(h)))
        return Connections(self, h, slot, dets)

    def build_target(self, conn: Connections, p_dets, validate=True) -> Connections:
        """The target set T = [V; P] of conn's V and the determinants p_dets (proxy matrix
        of Eq. 8); energy_and_grad on it evaluates the Proxy or Asymmetric objective."""
        p_dets = _dev_tensor(p_dets, torch.int64, "p_dets", self.device)
        h = C.c_void_p()
        self._check(lib().dnqs_build_target(self.handle, conn.slot, conn.handle, _ptr(p_dets), p_dets.shape[0],
                                            VALIDATE if validate else 0, C.byref(h)))
        T = torch.cat([conn.dets, p_dets], dim=0)
        c = Connections(self, h, conn.slot, T)
        c.n_v = conn.n
        return c

    def param_count(self, widths, slot=0):
        M, na, nb = self._slots[slot]
        return int(lib().dnqs_param_count(C.byref(Net.from_widths(widths)), M, na, nb))

    def amplitudes(self, widths, theta, dets, slot=0, precision=FP32):
        theta = _dev_tensor(theta, torch.float32, "theta", self.device)
        dets = _dev_tensor(dets, torch.int64, "dets", self.device)
        if theta.numel() != self.param_count(widths, slot):
            raise ValueError("theta has the wrong size for this network")
        n = dets.shape[0]
        la = torch.empty(n, dtype=torch.float64, device=dets.device)
        sg = torch.empty(n, dtype=torch.int8, device=dets.device)
        net = Net.from_widths(widths)
        self._check(lib().dnqs_amplitudes(self.handle, slot, C.byref(net), _ptr(theta), _ptr(dets), n, precision,
                                          _ptr(la), _ptr(sg)))
        return la, sg

    def energy_and_grad(self, widths, theta, conn: Connections, want_grad=True, precision=FP32, keep=True,
                        full_output=False, mode="default", recompute=False):
        """mode: "default" (Eq. 11 on a set S; the Proxy objective on a target set), "asym"
        (Eq. 6 with its exact gradient) or "asym_estimator" (Eq. 6 with Eq. 7's estimator)."""
        theta = _dev_tensor(theta, torch.float32, "theta", self.device)
        if theta.numel() != self.param_count(widths, conn.slot):
            raise ValueError("theta has the wrong size for this network")
        dev = theta.device
        n = conn.n
        E = torch.empty(1, dtype=torch.float64, device=dev)
        stats = torch.empty(3, dtype=torch.float64, device=dev)
        grad = torch.empty_like(theta) if want_grad else None
        v = torch.empty(n, dtype=torch.float64, device=dev) if keep else None
        la = torch.empty(n, dtype=torch.float64, device=dev) if keep else None
        sg = torch.empty(n, dtype=torch.int8, device=dev) if keep else None
        net = Net.from_widths(widths)
        flags = (FULL_OUTPUT if full_output else 0) | {"default": 0, "asym": ASYM, "asym_estimator": ASYM_ESTIMATOR}[mode]
        flags |= RECOMPUTE if recompute else 0
        self._check(lib().dnqs_energy_and_grad(self.handle, conn.slot, C.byref(net), _ptr(theta), conn.handle,
                                               precision, flags, _ptr(E), _ptr(stats), _ptr(grad), _ptr(v), _ptr(la),
                                               _ptr(sg)))
        return {"E": E, "stats": stats, "grad": grad, "v": v, "logabs": la, "sign": sg}

    def pt2(self, conn: Connections, logabs, sign, energy, sample_mask=0, export_cap=0, max_pair_bytes=0,
            eps_hb=0.0):
        dev = energy.device
        logabs = _dev_tensor(logabs, torch.float64, "logabs", self.device)
        sign = _dev_tensor(sign, torch.int8, "sign", self.device)
        energy = _dev_tensor(energy, torch.float64, "energy", self.device)
        out = torch.empty(4, dtype=torch.float64, device=dev)
        counts = torch.empty(6, dtype=torch.int64, device=dev)
        opts = PT2Opts()
        opts.sample_mask = int(sample_mask)
        opts.max_pair_bytes = int(max_pair_bytes)
        opts.eps_hb = float(eps_hb)
        ex = None
        if export_cap > 0:
            ex = {"keys": torch.empty((export_cap, 2), dtype=torch.int64, device=dev),
                  "w": torch.empty(export_cap, dtype=torch.float64, device=dev),
                  "haa": torch.empty(export_cap, dtype=torch.float64, device=dev),
                  "count": torch.zeros(1, dtype=torch.int64, device=dev)}
            opts.export_cap = export_cap
            opts.export_keys = ex["keys"].data_ptr()
            opts.export_w = ex["w"].data_ptr()
            opts.export_haa = ex["haa"].data_ptr()
            opts.export_count = ex["count"].data_ptr()
        self._check(lib().dnqs_pt2(self.handle, conn.slot, conn.handle, _ptr(logabs), _ptr(sign), _ptr(energy),
                                   C.byref(opts), _ptr(out), _ptr(counts)))
        res = {"out": out, "counts": counts}
        if ex is not None:
            res["export"] = ex
        return res

    def lanczos(self, conn: Connections, max_iter=300, tol=1e-10, start=None, want_vec=True):
        """Lowest eigenpair of H_SS: {"E": dev float64[1], "vec": dev float64[n] or None,
        "iters": int, "residual": float}."""
        dev = f"cuda:{self.device}"
        E = torch.empty(1, dtype=torch.float64, device=dev)
        vec = torch.empty(conn.n, dtype=torch.float64, device=dev) if want_vec else None
        if start is not None:
            start = _dev_tensor(start, torch.float64, "start", self.device)
        it, res = C.c_int(), C.c_double()
        self._check(lib().dnqs_lanczos(self.handle, conn.handle, int(max_iter), float(tol), _ptr(start), _ptr(E),
                                       _ptr(vec), C.byref(it), C.byref(res)))
        return {"E": E, "vec": vec, "iters": it.value, "residual": res.value}

    def heatbath_candidates(self, conn: Connections, logabs, sign, eps_hb, cap=None):
        """The screened perturbative set P_k (Eq. 14) as a dev int64[|P_k|, 2] tensor
        in canonical order."""
        logabs = _dev_tensor(logabs, torch.float64, "logabs", self.device)
        sign = _dev_tensor(sign, torch.int8, "sign", self.device)
        cap = int(cap) if cap is not None else 1 << 20
        while True:
            out = torch.empty((max(cap, 1), 2), dtype=torch.int64, device=logabs.device)
            n = C.c_int64()
            self._check(lib().dnqs_heatbath_candidates(self.handle, conn.slot, conn.handle, _ptr(logabs), _ptr(sign),
                                                       float(eps_hb), cap, _ptr(out), C.byref(n)))
            if n.value <= cap:
                return out[: n.value]
            cap = n.value

    def select_topk(self, dets, logabs, sign, K, slot=0):
        """The min(K, n) determinants of dets with the largest |psi| (ties: lower first),
        in canonical order (dev int64[k, 2])."""
        dets = _dev_tensor(dets, torch.int64, "dets", self.device)
        logabs = _dev_tensor(logabs, torch.float64, "logabs", self.device)
        if sign is not None:
            sign = _dev_tensor(sign, torch.int8, "sign", self.device)
        n = dets.shape[0]
        out = torch.empty((max(min(n, K), 1), 2), dtype=torch.int64, device=dets.device)
        k = C.c_int64()
        self._check(lib().dnqs_select_topk(self.handle, slot, _ptr(dets), _ptr(logabs), _ptr(sign), n, int(K),
                                           _ptr(out), C.byref(k)))
        return out[: k.value]

    # -------------------------------------------------------------- batched geometries
    def batch(self, widths, slots, conns, thetas, want_grad=True):
        """Device buffers and the C problem table for a batch (one entry per geometry)."""
        dev = thetas[0].device
        G = len(conns)
        probs = (Problem * G)()
        keep = []
        for g in range(G):
            th = _dev_tensor(thetas[g], torch.float32, "theta", self.device)
            E = torch.empty(1, dtype=torch.float64, device=dev)
            st = torch.empty(3, dtype=torch.float64, device=dev)
            gr = torch.empty_like(th) if want_grad else None
            probs[g].slot = slots[g]
            probs[g].conn = conns[g].handle
            probs[g].theta = th.data_ptr()
            probs[g].grad = gr.data_ptr() if gr is not None else None
            probs[g].energy = E.data_ptr()
            probs[g].stats = st.data_ptr()
            keep.append({"theta": th, "E": E, "stats": st, "grad": gr})
        return {"widths": tuple(widths), "probs": probs, "buffers": keep, "conns": conns}

    def energy_and_grad_batched(self, batch, precision=FP32):
        net = Net.from_widths(batch["widths"])
        self._check(lib().dnqs_energy_and_grad_batched(self.handle, C.byref(net), len(batch["buffers"]),
                                                       batch["probs"], precision, 0))
        return batch["buffers"]

    def adamw_batched(self, batch, m, v, step, lr_max=1e-3, lr_min=5e-5, decay_steps=800, beta1=0.9, beta2=0.999,
                      eps=1e-8, weight_decay=1e-2):
        cfg = AdamwCfg(lr_max, lr_min, decay_steps, beta1, beta2, eps, weight_decay)
        net = Net.from_widths(batch["widths"])
        self._check(lib().dnqs_adamw_batched(self.handle, C.byref(net), len(batch["buffers"]), batch["probs"],
                                             _ptr(m), _ptr(v), C.byref(cfg), _ptr(step)))

    def capture_begin(self):
        self._check(lib().dnqs_capture_begin(self.handle))

    def capture_end(self):
        g = C.c_void_p()
        self._check(lib().dnqs_capture_end(self.handle, C.byref(g)))
        return Graph(self, g)

    # -------------------------------------------------------------- timing
    def autotune(self, on=True):
        """Time the GEMM tile candidates of each new shape on first use (see dnqs.h)."""
        self._check(lib().dnqs_autotune(self.handle, 1 if on else 0))

    def tune_export(self) -> str:
        n = lib().dnqs_tune_export(self.handle, None, 0)
        buf = C.create_string_buffer(n + 1)
        lib().dnqs_tune_export(self.handle, buf, n + 1)
        return buf.value.decode()

    def tune_import(self, text: str):
        self._check(lib().dnqs_tune_import(self.handle, text.encode()))

    def timing(self, on=True):
        self._check(lib().dnqs_timing_enable(self.handle, 1 if on else 0))

    def timing_reset(self):
        self._check(lib().dnqs_timing_reset(self.handle))

    def timing_get(self, family):
        ms, k = C.c_double(), C.c_int64()
        self._check(lib().dnqs_timing_get(self.handle, family.encode(), C.byref(ms), C.byref(k)))
        return ms.value, k.value


class Graph:
    """A captured sequence of library calls, replayed on the context's stream."""

    def __init__(self, ctx, handle):
        self._ctx = ctx
        self.handle = handle
        _open_objects.add(self)

    def launch(self):
        self._ctx._check(lib().dnqs_graph_launch(self._ctx.handle, self.handle))

    def free(self):
        if self.handle:
            lib().dnqs_graph_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def dets_to_device(dets_np, device=0):
    """uint64[n,2] numpy -> int64 CUDA tensor with the same bits."""
    a = np.ascontiguousarray(np.asarray(dets_np, dtype=np.uint64).reshape(-1, 2)).view(np.int64)
    return torch.from_numpy(a.copy()).to(f"cuda:{device}")


def dets_to_host(dets_t):
    return dets_t.detach().cpu().numpy().view(np.uint64).reshape(-1, 2)


class DetNQSEnergy(torch.autograd.Function):
    """E(theta) of Eq. 11 with the library's adjoint (Eq. 12) as its backward."""

    @staticmethod
    def forward(ctx, theta, dctx: Context, widths, conn: Connections, precision=FP32):
        res = dctx.energy_and_grad(widths, theta.detach().contiguous(), conn, want_grad=True, precision=precision,
                                   keep=False)
        ctx.save_for_backward(res["grad"])
        return res["E"][0]

    @staticmethod
    def backward(ctx, gE):
        (grad,) = ctx.saved_tensors
        return (gE.to(grad.dtype) * grad, None, None, None, None)
