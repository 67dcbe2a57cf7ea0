"""Marshalling conveniences over the C ABI: a system with its built-in program,
spawning, composing, sending and receiving with numpy arrays or torch tensors.

Nothing here computes: every call goes through ``libka.so``.
"""
from __future__ import annotations

import ctypes
from ctypes import byref, c_void_p

import numpy as np

from . import (ka_wah_batch_result, KA_IN, KA_IN_OUT, KA_OUT, KA_PRIV, KA_REF, KA_SYS_PROFILE, KA_U32, KA_VAL, KA_WAH_INPUT_DEVICE, KA_WAH_VALUE_BITS,
               KA_WAH_OUTPUT_REFS, arg, check, ka_nd_range, ka_system_config, ka_value, ka_wah_result, lib,
               nd_range, ref, sig, val, values)


class Session:
    """One kernel-actor system on device 0 plus its built-in program."""

    def __init__(self, n_streams: int = 1, profile: bool = False, budget_bytes: int = 0,
                 use_torch_stream: bool = True):
        cfg = ka_system_config()
        cfg.device = 0
        cfg.n_streams = n_streams
        cfg.hbm_budget_bytes = budget_bytes
        cfg.flags = KA_SYS_PROFILE if profile else 0
        self.torch_stream = None
        if use_torch_stream:
            # A dedicated stream (default priority) made torch's current one, so
            # torch copies, torch events and the library's kernels are ordered.
            import torch
            self.torch_stream = torch.cuda.Stream()
            torch.cuda.set_stream(self.torch_stream)
            cfg.stream = self.torch_stream.cuda_stream
        self.sys = c_void_p()
        check(lib.ka_system_create(byref(cfg), byref(self.sys)), "ka_system_create")
        self.prog = c_void_p()
        check(lib.ka_program_builtin(self.sys, byref(self.prog)), "ka_program_builtin")
        self._keep = []

    # ---- actors --------------------------------------------------------------------
    def spawn(self, kernel: str, args, rng: ka_nd_range | None = None, prog=None) -> c_void_p:
        a = c_void_p()
        s = sig(*args)
        r = rng if rng is not None else nd_range()
        check(lib.ka_spawn(self.sys, prog or self.prog, kernel.encode(), byref(r), s, len(args), byref(a)),
              f"ka_spawn {kernel}")
        return a

    def compose(self, outer, inner) -> c_void_p:
        c = c_void_p()
        check(lib.ka_compose(outer, inner, byref(c)), "ka_compose")
        return c

    def release_actor(self, a):
        check(lib.ka_actor_release(a), "ka_actor_release")

    def affine_actor(self, a: int, b: int, in_mode=KA_REF, out_mode=KA_REF) -> c_void_p:
        ca = (ctypes.c_uint32 * 1)(a)
        cb = (ctypes.c_uint32 * 1)(b)
        return self.spawn("affine_u32", [arg(KA_IN_OUT, in_mode=in_mode, out_mode=out_mode),
                                         arg(KA_PRIV, count=1, init=ca), arg(KA_PRIV, count=1, init=cb)])

    # ---- messages ------------------------------------------------------------------
    def send(self, actor, *vs: ka_value) -> c_void_p:
        t = c_void_p()
        check(lib.ka_send(actor, values(*vs) if vs else None, len(vs), byref(t)), "ka_send")
        return t

    def receive(self, ticket, n: int, timeout_us: int = -1):
        """Receives n outputs: REF outputs as refs, VAL outputs as numpy arrays."""
        outs = (ka_value * n)()
        check(lib.ka_receive(ticket, outs, n, timeout_us), "ka_receive")  # sizes / refs
        res = []
        for i in range(n):
            if outs[i].mode == KA_REF:
                res.append(c_void_p(outs[i].ref))
            else:
                buf = np.empty(outs[i].count, dtype=np.uint32)
                res.append(buf)
        vals = [i for i in range(n) if outs[i].mode == KA_VAL]
        if vals:
            outs2 = (ka_value * n)()
            for i in range(n):
                if i in vals:
                    outs2[i].ptr = res[i].ctypes.data if res[i].size else None
                    outs2[i].count = res[i].size
            check(lib.ka_receive(ticket, outs2, n, timeout_us), "ka_receive")
            for i in range(n):
                if outs2[i].mode == KA_REF:  # the second receive returned new refs too
                    lib.ka_ref_release(c_void_p(outs2[i].ref))
        return res

    def release_ticket(self, t):
        check(lib.ka_ticket_release(t), "ka_ticket_release")

    def request(self, actor, *vs: ka_value, n_out: int):
        t = self.send(actor, *vs)
        try:
            return self.receive(t, n_out)
        finally:
            self.release_ticket(t)

    def batch_run(self, actor, requests):
        """ka_batch_run: requests is a list of messages (each a list of
        ka_value); returns one ticket per request."""
        from . import ka_request
        n = len(requests)
        msgs = [values(*m) for m in requests]  # kept alive until the call returns
        reqs = (ka_request * max(n, 1))()
        for i, m in enumerate(msgs):
            reqs[i].args = ctypes.cast(m, ctypes.POINTER(ka_value))
            reqs[i].nargs = len(requests[i])
        tickets = (c_void_p * max(n, 1))()
        check(lib.ka_batch_run(actor, reqs, n, tickets), "ka_batch_run")
        return [c_void_p(tickets[i]) for i in range(n)]

    # ---- refs ----------------------------------------------------------------------
    def wrap(self, tensor) -> c_void_p:
        """Borrowed ref over a contiguous 4-byte torch tensor on the device."""
        assert tensor.is_cuda and tensor.is_contiguous() and tensor.element_size() == 4
        r = c_void_p()
        check(lib.ka_ref_wrap(self.sys, c_void_p(tensor.data_ptr()), KA_U32, tensor.numel(), 3, byref(r)),
              "ka_ref_wrap")
        return r

    def upload(self, x: np.ndarray):
        """A torch tensor on the device holding the uint32 array x."""
        import torch
        x = np.ascontiguousarray(x, dtype=np.uint32)
        return torch.from_numpy(x.view(np.int32)).to("cuda")

    def length(self, r) -> int:
        n = ctypes.c_uint64()
        check(lib.ka_ref_info(r, None, byref(n), None), "ka_ref_info")
        return n.value

    def read(self, r) -> np.ndarray:
        n = self.length(r)
        out = np.empty(n, dtype=np.uint32)
        if n:
            check(lib.ka_ref_read(r, out.ctypes.data, n * 4), "ka_ref_read")
        return out

    def release_ref(self, r):
        check(lib.ka_ref_release(r), "ka_ref_release")

    def device_ptr(self, r) -> int:
        p = c_void_p()
        check(lib.ka_ref_device_ptr(r, byref(p)), "ka_ref_device_ptr")
        return p.value or 0

    # ---- composed index --------------------------------------------------------------
    def wah_index(self, values_, refs: bool = False, value_bits: int = 0, fmt: int = 0):
        """WAH index of a numpy uint32 array (host input) or a device tensor.
        value_bits: every value is below 2^value_bits (0: no hint); fmt: word
        format (0 paper, 1 canonical, 2 PLWAH).
        Returns (keys, offsets, words) numpy arrays, or the result struct with refs."""
        from . import KA_WAH_FORMAT
        res = ka_wah_result()
        flags = (KA_WAH_OUTPUT_REFS if refs else 0) | KA_WAH_VALUE_BITS(value_bits) | KA_WAH_FORMAT(fmt)
        if isinstance(values_, np.ndarray):
            v = np.ascontiguousarray(values_, dtype=np.uint32)
            check(lib.ka_wah_index(self.sys, v.ctypes.data if v.size else None, v.size, flags, byref(res)),
                  "ka_wah_index")
        else:
            check(lib.ka_wah_index(self.sys, c_void_p(values_.data_ptr()), values_.numel(),
                                   flags | KA_WAH_INPUT_DEVICE, byref(res)), "ka_wah_index")
        if refs:
            return res
        D, W = res.D, res.W
        keys = np.ctypeslib.as_array(res.keys, shape=(max(D, 1),))[:D].copy()
        offs = np.ctypeslib.as_array(res.offsets, shape=(D + 1,)).copy()
        words = np.ctypeslib.as_array(res.words, shape=(max(W, 1),))[:W].copy()
        check(lib.ka_wah_result_free(byref(res)), "ka_wah_result_free")
        return keys, offs, words

    def wah_batch(self, values_, req_off, value_bits: int, refs: bool = False):
        """Index of every request of a batch (ka_wah_batch).  values_: numpy
        uint32 array (host) or device tensor of the concatenated requests;
        req_off: nreq + 1 request boundaries.  Returns a list of per-request
        (keys, offsets, words), or the result struct with refs."""
        off = np.ascontiguousarray(req_off, dtype=np.uint32)
        nreq = off.size - 1
        res = ka_wah_batch_result()
        flags = KA_WAH_OUTPUT_REFS if refs else 0
        if isinstance(values_, np.ndarray):
            v = np.ascontiguousarray(values_, dtype=np.uint32)
            check(lib.ka_wah_batch(self.sys, v.ctypes.data if v.size else None, v.size, off.ctypes.data, nreq,
                                   value_bits, flags, byref(res)), "ka_wah_batch")
        else:
            check(lib.ka_wah_batch(self.sys, c_void_p(values_.data_ptr()), values_.numel(), off.ctypes.data, nreq,
                                   value_bits, flags | KA_WAH_INPUT_DEVICE, byref(res)), "ka_wah_batch")
        if refs:
            return res
        D, W = res.D, res.W
        keys = np.ctypeslib.as_array(res.keys, shape=(max(D, 1),))[:D].copy()
        offs = np.ctypeslib.as_array(res.offsets, shape=(D + nreq,)).copy()
        words = np.ctypeslib.as_array(res.words, shape=(max(W, 1),))[:W].copy()
        ks = np.ctypeslib.as_array(res.key_start, shape=(nreq + 1,)).copy()
        ws = np.ctypeslib.as_array(res.word_start, shape=(nreq + 1,)).copy()
        check(lib.ka_wah_batch_result_free(byref(res)), "ka_wah_batch_result_free")
        out = []
        for j in range(nreq):
            k0, k1, w0, w1 = int(ks[j]), int(ks[j + 1]), int(ws[j]), int(ws[j + 1])
            out.append((keys[k0:k1], offs[k0 + j:k1 + j + 1], words[w0:w1]))
        return out

    def stream_handle(self, i: int = 0) -> int:
        s = c_void_p()
        check(lib.ka_system_stream(self.sys, i, byref(s)), "ka_system_stream")
        return s.value or 0

    def synchronize(self):
        check(lib.ka_system_synchronize(self.sys), "ka_system_synchronize")

    def profile(self, kernel: str):
        n = ctypes.c_uint64()
        ms = ctypes.c_double()
        check(lib.ka_profile_get(self.sys, kernel.encode(), byref(n), byref(ms)), "ka_profile_get")
        return n.value, ms.value

    def profile_reset(self):
        check(lib.ka_profile_reset(self.sys), "ka_profile_reset")

    def memory(self):
        a, b = ctypes.c_uint64(), ctypes.c_uint64()
        check(lib.ka_system_memory(self.sys, byref(a), byref(b)), "ka_system_memory")
        return a.value, b.value

    def length_reads(self):
        """Device-resident lengths read back on the host so far."""
        c = ctypes.c_uint64()
        check(lib.ka_system_length_reads(self.sys, byref(c)), "ka_system_length_reads")
        return c.value

    def close(self):
        if self.prog:
            lib.ka_program_release(self.prog)
            self.prog = None
        if self.sys:
            check(lib.ka_system_destroy(self.sys), "ka_system_destroy")
            self.sys = None
        if self.torch_stream is not None:
            import torch
            torch.cuda.synchronize()
            torch.cuda.set_stream(torch.cuda.default_stream())
            self.torch_stream = None


def sig_in(mode=KA_REF):
    return arg(KA_IN, in_mode=mode)


def sig_out(mode=KA_REF, count=0):
    return arg(KA_OUT, out_mode=mode, count=count)


__all__ = ["Session", "sig_in", "sig_out", "val", "ref", "KA_VAL", "KA_REF"]


class Server:
    """The served form (ka_server_*): submit requests, wait for them, read
    their outputs and the latency statistics."""

    def __init__(self, session: Session, streams: int = 2, max_batch: int = 0, budget_bytes: int = 0,
                 value_bits: int = 12, chain_a=None, chain_b=None, max_batch_bytes: int = 0,
                 copy_threads: int = 0):
        from . import ka_server_config
        cfg = ka_server_config()
        cfg.copy_threads = copy_threads
        cfg.streams = streams
        cfg.max_batch = max_batch
        cfg.max_batch_bytes = max_batch_bytes
        cfg.hbm_budget_bytes = budget_bytes
        cfg.value_bits = value_bits
        self._a = np.ascontiguousarray(chain_a if chain_a is not None else [], dtype=np.uint32)
        self._b = np.ascontiguousarray(chain_b if chain_b is not None else [], dtype=np.uint32)
        cfg.chain_len = self._a.size
        if self._a.size:
            cfg.chain_a = self._a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
            cfg.chain_b = self._b.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
        self.srv = c_void_p()
        check(lib.ka_server_create(session.sys, byref(cfg), byref(self.srv)), "ka_server_create")

    @staticmethod
    def clock_us() -> float:
        t = ctypes.c_double()
        check(lib.ka_server_clock_us(byref(t)), "ka_server_clock_us")
        return t.value

    def submit(self, kind: int, data: np.ndarray, arrival_us: float = 0.0):
        d = np.ascontiguousarray(data, dtype=np.uint32)
        r = c_void_p()
        check(lib.ka_server_submit(self.srv, kind, d.ctypes.data if d.size else None, d.size, arrival_us, byref(r)),
              "ka_server_submit")
        return r

    def send(self, kind: int, data, refs: bool = False, arrival_us: float = 0.0):
        """ka_server_send: data is a numpy uint32 array (a host value) or a
        ka_ref handle (a device reference); returns the ticket."""
        from . import KA_SRV_OUTPUT_REFS
        if isinstance(data, np.ndarray):
            d = np.ascontiguousarray(data, dtype=np.uint32)
            v = val(d.ctypes.data if d.size else None, d.size)
        else:
            v = ref(data)
        t = c_void_p()
        check(lib.ka_server_send(self.srv, kind, byref(v), 1, KA_SRV_OUTPUT_REFS if refs else 0, arrival_us,
                                 byref(t)), "ka_server_send")
        return t

    def wait(self, req, timeout_us: int = -1) -> int:
        return lib.ka_server_wait(req, timeout_us)

    def result(self, req, i: int = 0) -> np.ndarray:
        n = ctypes.c_uint64()
        check(lib.ka_server_result(req, i, None, 0, byref(n)), "ka_server_result")
        out = np.empty(n.value, dtype=np.uint32)
        check(lib.ka_server_result(req, i, out.ctypes.data if out.size else None, out.size, byref(n)),
              "ka_server_result")
        return out

    def release(self, req):
        check(lib.ka_server_request_release(req), "ka_server_request_release")

    def stats(self):
        from . import ka_server_stats
        st = ka_server_stats()
        check(lib.ka_server_get_stats(self.srv, byref(st)), "ka_server_get_stats")
        return {f: getattr(st, f) for f, _ in st._fields_}

    def reset_stats(self):
        check(lib.ka_server_reset_stats(self.srv), "ka_server_reset_stats")

    def close(self):
        if self.srv:
            check(lib.ka_server_destroy(self.srv), "ka_server_destroy")
            self.srv = None


class BatchPlan:
    """A batch shape recorded into a HIP graph (ka_batch_plan_*)."""

    def __init__(self, session: Session, req_off, value_bits: int, autotune: bool = False, shape: int | None = None,
                 any_batch=None):
        """req_off: the one batch shape; or any_batch = (max_values,
        max_requests, max_request_values) for a plan that serves any batch
        within these capacities (req_off then ignored, may be None)."""
        self.plan = c_void_p()
        flags = (1 if autotune else 0) | (((shape + 1) << 8) if shape is not None else 0)
        if any_batch is not None:
            mv, mr, mq = any_batch
            check(lib.ka_batch_plan_create_any(session.sys, mv, mr, mq, value_bits, flags, byref(self.plan)),
                  "ka_batch_plan_create_any")
            return
        self.off = np.ascontiguousarray(req_off, dtype=np.uint32)
        check(lib.ka_batch_plan_create(session.sys, self.off.ctypes.data, self.off.size - 1, value_bits, flags,
                                       byref(self.plan)), "ka_batch_plan_create")

    def shape(self):
        """(shape used by the runs, first-run times per shape in ms)."""
        sh = ctypes.c_int()
        ms = (ctypes.c_float * 4)()
        check(lib.ka_batch_plan_shape(self.plan, byref(sh), ms, 4), "ka_batch_plan_shape")
        return sh.value, list(ms)

    def stream_handle(self) -> int:
        s = c_void_p()
        check(lib.ka_batch_plan_stream(self.plan, byref(s)), "ka_batch_plan_stream")
        return s.value or 0

    def input_ptr(self) -> int:
        p = c_void_p()
        check(lib.ka_batch_plan_input(self.plan, byref(p)), "ka_batch_plan_input")
        return p.value or 0

    def run(self, values=None):
        """values: numpy uint32 (host), a device tensor, or None (input buffer already filled)."""
        if values is None:
            check(lib.ka_batch_plan_run(self.plan, None, 0), "ka_batch_plan_run")
        elif isinstance(values, np.ndarray):
            v = np.ascontiguousarray(values, dtype=np.uint32)
            check(lib.ka_batch_plan_run(self.plan, v.ctypes.data if v.size else None, 0), "ka_batch_plan_run")
        else:
            check(lib.ka_batch_plan_run(self.plan, c_void_p(values.data_ptr()), KA_WAH_INPUT_DEVICE),
                  "ka_batch_plan_run")

    def run_batch(self, values, req_off):
        """Any-batch plans: the next batch (values: numpy uint32 on the host or
        a device tensor; req_off: nreq + 1 entries)."""
        off = np.ascontiguousarray(req_off, dtype=np.uint32)
        if isinstance(values, np.ndarray):
            v = np.ascontiguousarray(values, dtype=np.uint32)
            ptr, fl = (v.ctypes.data if v.size else None), 0
        else:
            v, ptr, fl = values, c_void_p(values.data_ptr()), KA_WAH_INPUT_DEVICE
        check(lib.ka_batch_plan_run_batch(self.plan, ptr, off.ctypes.data, off.size - 1, fl),
              "ka_batch_plan_run_batch")

    def result(self):
        """Per-request (keys, offsets, words) of the last run."""
        res = ka_wah_batch_result()
        check(lib.ka_batch_plan_result(self.plan, byref(res)), "ka_batch_plan_result")
        nreq, D, W = res.nreq, res.D, res.W
        keys = np.ctypeslib.as_array(res.keys, shape=(max(D, 1),))[:D].copy()
        offs = np.ctypeslib.as_array(res.offsets, shape=(D + nreq,)).copy()
        words = np.ctypeslib.as_array(res.words, shape=(max(W, 1),))[:W].copy()
        ks = np.ctypeslib.as_array(res.key_start, shape=(nreq + 1,)).copy()
        ws = np.ctypeslib.as_array(res.word_start, shape=(nreq + 1,)).copy()
        check(lib.ka_wah_batch_result_free(byref(res)), "ka_wah_batch_result_free")
        return [(keys[ks[j]:ks[j + 1]], offs[ks[j] + j:ks[j + 1] + j + 1], words[ws[j]:ws[j + 1]])
                for j in range(nreq)]

    def close(self):
        if self.plan:
            check(lib.ka_batch_plan_destroy(self.plan), "ka_batch_plan_destroy")
            self.plan = None

