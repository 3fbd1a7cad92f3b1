"""Python binding of libgt.so: stable CSR -> CSC graph transposition on MI355X.

Argument marshalling only.  Every step of the transposition runs in the HIP
kernels of ``libgt.so``; PyTorch provides device memory and the stream.  If
the library has not been built, importing works but every call raises.

    T, S, Q = transpose(offsets, indices, payload=None)

``offsets`` int64[n+1], ``indices`` int32[m], ``payload`` a 32-bit tensor
(int32/uint32/float32, moved as bit patterns) or None, all on one GPU.
Returns the CSC offsets (int64[n+1]), sources (int32[m]) and payload
(same dtype as given, or None).
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgt.so")

(GT_OK, GT_ERR_INVALID_ARGUMENT, GT_ERR_INVALID_GRAPH, GT_ERR_WORKSPACE_TOO_SMALL, GT_ERR_UNSUPPORTED, GT_ERR_HIP,
 GT_ERR_COUNTER_OVERFLOW, GT_ERR_STALLED) = range(8)
MAX_EDGES = 1 << 32
NOALLOC_SCRATCH_BYTES = 64 << 20  # the library's own scratch per GPU (gt_transpose_noalloc)
POLICY_HEURISTIC, POLICY_FIXED, POLICY_MLP = range(3)
# STABLE: every CSC list in CSR edge order.  HLH / ATOMIC: the paper's methods,
# list order left to the atomics (offsets and list contents exact).
STRATEGY_STABLE, STRATEGY_HLH, STRATEGY_ATOMIC, STRATEGY_PROBE = range(4)

# Every entry point declared in include/gt.h.
EXPORTS = ("gt_workspace_size", "gt_plan_scratch_size", "gt_plan_workspace_size", "gt_plan", "gt_transpose",
           "gt_transpose_batched", "gt_transpose_noalloc", "gt_plan_device_status", "gt_device_status", "gt_plan_params",
           "gt_plan_device_choice", "gt_plan_packed", "gt_plan_strategy",
           "gt_plan_step3_times", "gt_plan_destroy", "gt_profile", "gt_profile_read", "gt_plan_features", "gt_config",
           "gt_autotune", "gt_plan_set_config", "gt_mlp_forward", "gt_mlp_gradient", "gt_mlp_adam",
           "gt_random_access", "gt_num_configs", "gt_mlp_num_params", "gt_mlp_work_floats", "gt_status_string")
NUM_FEATURES = 16


class GTError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})")


class CSR(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("offsets", ctypes.c_void_p),
                ("indices", ctypes.c_void_p), ("payload", ctypes.c_void_p)]


class CSC(ctypes.Structure):
    _fields_ = [("offsets", ctypes.c_void_p), ("indices", ctypes.c_void_p), ("payload", ctypes.c_void_p)]


class Options(ctypes.Structure):
    _fields_ = [("policy", ctypes.c_int32), ("fine_bits", ctypes.c_int32), ("digit_bits", ctypes.c_int32),
                ("variant", ctypes.c_int32), ("validate", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("model_path", ctypes.c_char_p), ("flags", ctypes.c_int32), ("strategy", ctypes.c_int32),
                ("hdv_max", ctypes.c_int32)]


_lib = None


def lib():
    """Load libgt.so (raises if it has not been built: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2501_06872_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
        P = ctypes.POINTER
        L.gt_workspace_size.argtypes = [P(CSR), i32, P(sz)]
        L.gt_plan_scratch_size.argtypes = [P(CSR), i32, P(sz)]
        L.gt_plan_workspace_size.argtypes = [vp, P(sz)]
        L.gt_plan.argtypes = [P(CSR), i32, P(Options), vp, sz, vp, P(vp)]
        L.gt_transpose.argtypes = [vp, P(CSR), P(CSC), vp, sz, vp]
        L.gt_transpose_batched.argtypes = [vp, i32, P(CSR), P(CSC), vp, sz, vp]
        L.gt_transpose_noalloc.argtypes = [vp, P(CSR), P(CSC), vp, vp]
        L.gt_device_status.argtypes = [vp]
        L.gt_plan_device_status.argtypes = [vp, vp]
        L.gt_plan_params.argtypes = [vp, i32, P(i32), P(i32), P(i32), P(i32)]
        L.gt_plan_device_choice.argtypes = [vp, vp, i32, P(i32), P(i32), P(i32), P(i32)]
        L.gt_plan_strategy.argtypes = [vp, i32, P(i32)]
        L.gt_plan_packed.argtypes = [vp, i32, P(i32)]
        L.gt_plan_destroy.argtypes = [vp]
        L.gt_plan_step3_times.argtypes = [vp, i32, vp, vp, i32, P(i32), P(ctypes.c_double)]
        L.gt_profile.argtypes = [vp, i32]
        L.gt_profile_read.argtypes = [vp, i32, vp, vp, vp, P(i32)]
        L.gt_plan_features.argtypes = [vp, i32, vp, i32, P(i32)]
        L.gt_config.argtypes = [i32, P(i32), P(i32), P(i32)]
        L.gt_autotune.argtypes = [P(CSR), P(CSC), vp, sz, vp, i32, vp]
        L.gt_plan_set_config.argtypes = [vp, i32, i32]
        L.gt_mlp_forward.argtypes = [vp, vp, i32, vp, vp]
        L.gt_mlp_gradient.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp, vp]
        fl = ctypes.c_float
        L.gt_mlp_adam.argtypes = [vp, vp, vp, vp, i32, fl, fl, fl, fl, vp]
        L.gt_random_access.argtypes = [vp, ctypes.c_uint64, i32, i32, ctypes.c_uint32, ctypes.c_int64, i32, vp, vp]
        L.gt_num_configs.argtypes = []
        L.gt_mlp_num_params.argtypes = []
        L.gt_mlp_work_floats.argtypes = [i32]
        L.gt_mlp_work_floats.restype = ctypes.c_size_t
        L.gt_status_string.argtypes = [ctypes.c_int]
        L.gt_status_string.restype = ctypes.c_char_p
        for f in EXPORTS[:-2]:
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def status_string(s):
    return lib().gt_status_string(int(s)).decode()


def _check(rc, what):
    if rc != GT_OK:
        raise GTError(rc, what)


def _stream_ptr(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _csr(offsets, indices, payload):
    n = offsets.numel() - 1
    m = indices.numel()
    return CSR(n, m, offsets.data_ptr(), indices.data_ptr() if m else None,
               payload.data_ptr() if payload is not None and m else (1 if payload is not None else None))


def _check_inputs(offsets, indices, payload):
    if not (offsets.is_cuda and indices.is_cuda):
        raise ValueError("offsets and indices must be GPU tensors")
    if offsets.dtype != torch.int64 or indices.dtype != torch.int32:
        raise ValueError("offsets must be int64 and indices int32")
    if not (offsets.is_contiguous() and indices.is_contiguous()):
        raise ValueError("inputs must be contiguous")
    if payload is not None:
        if payload.element_size() != 4 or payload.numel() != indices.numel() or not payload.is_contiguous():
            raise ValueError("payload must be a contiguous 32-bit tensor with one word per edge")


(FLAG_WIDE_STATUS, FLAG_FEATURES, FLAG_STEP3_STATIC, FLAG_STEP3_STEAL, FLAG_STEP3_TIMES, FLAG_PERSISTENT,
 FLAG_DEVICE_PLAN) = 1, 2, 4, 8, 16, 32, 64


def make_options(policy=POLICY_HEURISTIC, fine_bits=0, digit_bits=0, variant=0, validate=False, seed=0,
                 model_path=None, flags=0, strategy=STRATEGY_STABLE, hdv_max=0):
    return Options(policy, fine_bits, digit_bits, variant, int(bool(validate)), seed,
                   model_path.encode() if model_path else None, flags, strategy, hdv_max)


class Plan:
    """A plan plus its workspace for graphs of fixed sizes.

    ``Plan([(offsets, indices, payload), ...], options)``; call ``run`` (one
    graph) or ``run_batched`` (all graphs) with tensors of the same sizes.
    """

    def __init__(self, graphs, options=None, device=None, workspace=None):
        L = lib()
        self.device = device if device is not None else graphs[0][0].device
        self.count = len(graphs)
        for g in graphs:
            _check_inputs(*g)
        arr = (CSR * self.count)(*[_csr(*g) for g in graphs])
        self._shapes = [(g[0].numel() - 1, g[1].numel(), g[2] is not None) for g in graphs]
        # planning needs the sampling scratch only; the transposition needs
        # what the chosen parameters need (gt_plan_workspace_size)
        opts = options if options is not None else make_options()
        ws = ctypes.c_size_t(0)
        # the probe runs Step 1 in the transposition layout; a device plan
        # keeps its choices in the workspace the transpositions use
        if opts.strategy == STRATEGY_PROBE or (opts.flags & FLAG_DEVICE_PLAN):
            _check(L.gt_workspace_size(arr, self.count, ctypes.byref(ws)), "gt_workspace_size")
        else:
            _check(L.gt_plan_scratch_size(arr, self.count, ctypes.byref(ws)), "gt_plan_scratch_size")
        self.workspace = self._buffer(int(ws.value), workspace)
        h = ctypes.c_void_p()
        _check(L.gt_plan(arr, self.count, ctypes.byref(opts), self.workspace.data_ptr(), self.workspace.numel(),
                         _stream_ptr(self.device), ctypes.byref(h)), "gt_plan")
        self.handle = h
        self._fit_workspace(workspace)

    def _buffer(self, nbytes, given=None):
        if given is not None and given.numel() >= nbytes:
            return given
        if getattr(self, "workspace", None) is not None and self.workspace.numel() >= nbytes:
            return self.workspace
        return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)

    def workspace_size(self):
        ws = ctypes.c_size_t(0)
        _check(lib().gt_plan_workspace_size(self.handle, ctypes.byref(ws)), "gt_plan_workspace_size")
        return int(ws.value)

    def _fit_workspace(self, given=None):
        need = self.workspace_size()
        if self.workspace.numel() < need:
            self.workspace = None
            self.workspace = self._buffer(need, given)

    def params(self, i=0):
        a, b, c, d = (ctypes.c_int32() for _ in range(4))
        _check(lib().gt_plan_params(self.handle, i, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                    ctypes.byref(d)), "gt_plan_params")
        return dict(fine_bits=a.value, digit_bits=b.value, passes=c.value, variant=d.value)

    def device_choice(self, i=0):
        """GT_FLAG_DEVICE_PLAN plans: the parameters chosen on the device for
        graph i (synchronises on the copy)."""
        a, b, c, d = (ctypes.c_int32() for _ in range(4))
        _check(lib().gt_plan_device_choice(self.handle, self.workspace.data_ptr(), i, ctypes.byref(a),
                                           ctypes.byref(b), ctypes.byref(c), ctypes.byref(d)), "gt_plan_device_choice")
        return dict(fine_bits=a.value, digit_bits=b.value, variant=c.value, config=d.value)

    def packed(self, i=0):
        out = ctypes.c_int32()
        _check(lib().gt_plan_packed(self.handle, i, ctypes.byref(out)), "gt_plan_packed")
        return bool(out.value)

    def strategy(self, i=0):
        out = ctypes.c_int32()
        _check(lib().gt_plan_strategy(self.handle, i, ctypes.byref(out)), "gt_plan_strategy")
        return out.value

    def alloc_out(self, i=0, payload_dtype=torch.uint32):
        n, m, pay = self._shapes[i]
        T = torch.empty(n + 1, dtype=torch.int64, device=self.device)
        S = torch.empty(m, dtype=torch.int32, device=self.device)
        Q = torch.empty(m, dtype=payload_dtype, device=self.device) if pay else None
        return T, S, Q

    def run(self, offsets, indices, payload=None, out=None):
        _check_inputs(offsets, indices, payload)
        T, S, Q = out if out is not None else self.alloc_out(0, payload.dtype if payload is not None else None)
        g = _csr(offsets, indices, payload)
        o = CSC(T.data_ptr(), S.data_ptr() if S.numel() else None,
                (Q.data_ptr() if Q.numel() else 1) if Q is not None else None)
        _check(lib().gt_transpose(self.handle, ctypes.byref(g), ctypes.byref(o), self.workspace.data_ptr(),
                                  self.workspace.numel(), _stream_ptr(self.device)), "gt_transpose")
        return T, S, Q

    def run_noalloc(self, offsets, indices, payload, out, status=None):
        """gt_transpose_noalloc: the library's static scratch instead of the
        plan's workspace.  ``out`` = caller-allocated (T, S, Q); ``status``
        None or a 1-element 32-bit GPU tensor that receives the device
        status word."""
        _check_inputs(offsets, indices, payload)
        T, S, Q = out
        g = _csr(offsets, indices, payload)
        o = CSC(T.data_ptr(), S.data_ptr() if S.numel() else None,
                (Q.data_ptr() if Q.numel() else 1) if Q is not None else None)
        st = status.data_ptr() if status is not None else None
        _check(lib().gt_transpose_noalloc(self.handle, ctypes.byref(g), ctypes.byref(o), st,
                                          _stream_ptr(self.device)), "gt_transpose_noalloc")
        return T, S, Q

    def run_batched(self, graphs, outs=None):
        if outs is None:
            outs = [self.alloc_out(i, g[2].dtype if g[2] is not None else None) for i, g in enumerate(graphs)]
        arr = (CSR * self.count)(*[_csr(*g) for g in graphs])
        oarr = (CSC * self.count)(*[CSC(T.data_ptr(), S.data_ptr() if S.numel() else None,
                                        (Q.data_ptr() if Q.numel() else 1) if Q is not None else None)
                                    for T, S, Q in outs])
        _check(lib().gt_transpose_batched(self.handle, self.count, arr, oarr, self.workspace.data_ptr(),
                                          self.workspace.numel(), _stream_ptr(self.device)), "gt_transpose_batched")
        return outs

    def features(self, i=0):
        out = (ctypes.c_float * 32)()
        cnt = ctypes.c_int32()
        _check(lib().gt_plan_features(self.handle, i, out, 32, ctypes.byref(cnt)), "gt_plan_features")
        return [out[k] for k in range(min(cnt.value, 32))]

    def set_config(self, i, config):
        _check(lib().gt_plan_set_config(self.handle, i, config), "gt_plan_set_config")
        self._fit_workspace()

    def profile(self, enable=True):
        _check(lib().gt_profile(self.handle, int(bool(enable))), "gt_profile")

    def profile_read(self, max_kernels=32):
        """{kernel name: (total ms, launches)} since profiling was enabled or last read."""
        names = (ctypes.c_char * (32 * max_kernels))()
        ms = (ctypes.c_double * max_kernels)()
        nl = (ctypes.c_int32 * max_kernels)()
        cnt = ctypes.c_int32()
        _check(lib().gt_profile_read(self.handle, max_kernels, names, ms, nl, ctypes.byref(cnt)),
               "gt_profile_read")
        raw = bytes(names)
        out = {}
        for k in range(cnt.value):
            name = raw[32 * k: 32 * k + 32].split(b"\0", 1)[0].decode()
            out[name] = (ms[k], nl[k])
        return out

    def step3_times(self, i=0):
        """Per chunk workgroup of Step 3 (plans with FLAG_STEP3_TIMES):
        uint64 wall-clock stamps [start, own head done, end]."""
        import numpy as np
        torch.cuda.current_stream(self.device).synchronize()
        cnt = ctypes.c_int32()
        hz = ctypes.c_double()
        _check(lib().gt_plan_step3_times(self.handle, i, self.workspace.data_ptr(), None, 0, ctypes.byref(cnt),
                                         ctypes.byref(hz)), "gt_plan_step3_times")
        out = np.zeros((cnt.value, 3), dtype=np.uint64)
        _check(lib().gt_plan_step3_times(self.handle, i, self.workspace.data_ptr(), out.ctypes.data, cnt.value,
                                         ctypes.byref(cnt), ctypes.byref(hz)), "gt_plan_step3_times")
        self._step3_hz = hz.value
        return out

    def step3_clock_hz(self):
        return getattr(self, "_step3_hz", 100e6)

    def device_status(self):
        torch.cuda.current_stream(self.device).synchronize()
        return lib().gt_plan_device_status(self.handle, self.workspace.data_ptr())

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.gt_plan_destroy(h)
            self.handle = None


def workspace_bytes(graphs):
    """Workspace bytes for a list of (offsets, indices, payload) graphs."""
    arr = (CSR * len(graphs))(*[_csr(*g) for g in graphs])
    ws = ctypes.c_size_t(0)
    _check(lib().gt_workspace_size(arr, len(graphs), ctypes.byref(ws)), "gt_workspace_size")
    return int(ws.value)


def transpose(offsets, indices, payload=None, options=None):
    """Transpose one CSR graph on its GPU; returns (T, S, Q)."""
    plan = Plan([(offsets, indices, payload)], options)
    return plan.run(offsets, indices, payload)


def num_configs():
    return lib().gt_num_configs()


def config(idx):
    a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().gt_config(idx, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), "gt_config")
    return dict(fine_bits=a.value, digit_bits=b.value, variant=c.value)


def autotune(offsets, indices, payload=None, reps=5, plan=None):
    """Time every configuration (milliseconds, median of `reps`) on this graph."""
    _check_inputs(offsets, indices, payload)
    plan = plan if plan is not None else Plan([(offsets, indices, payload)], make_options(policy=POLICY_FIXED))
    T, S, Q = plan.alloc_out(0, payload.dtype if payload is not None else None)
    g = _csr(offsets, indices, payload)
    ws = ctypes.c_size_t(0)  # every configuration: the any-parameters bound
    _check(lib().gt_workspace_size(ctypes.byref(g), 1, ctypes.byref(ws)), "gt_workspace_size")
    plan.workspace = plan._buffer(int(ws.value))
    o = CSC(T.data_ptr(), S.data_ptr() if S.numel() else None,
            (Q.data_ptr() if Q.numel() else 1) if Q is not None else None)
    ms = (ctypes.c_float * num_configs())()
    _check(lib().gt_autotune(ctypes.byref(g), ctypes.byref(o), plan.workspace.data_ptr(), plan.workspace.numel(),
                             _stream_ptr(plan.device), reps, ms), "gt_autotune")
    return [ms[k] for k in range(num_configs())], (T, S, Q)


# ---- training primitives of the parameter-choice MLP (torch float32 tensors on one GPU)
def mlp_num_params():
    return lib().gt_mlp_num_params()


def mlp_forward(params, x):
    y = torch.empty((x.shape[0], 32), dtype=torch.float32, device=x.device)
    _check(lib().gt_mlp_forward(params.data_ptr(), x.data_ptr(), x.shape[0], y.data_ptr(), _stream_ptr(x.device)),
           "gt_mlp_forward")
    return y


def mlp_gradient(params, x, target, work=None):
    B = x.shape[0]
    y = torch.empty((B, 32), dtype=torch.float32, device=x.device)
    g = torch.empty_like(params)
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    if work is None:
        work = torch.empty(lib().gt_mlp_work_floats(B), dtype=torch.float32, device=x.device)
    _check(lib().gt_mlp_gradient(params.data_ptr(), x.data_ptr(), target.data_ptr(), B, y.data_ptr(), g.data_ptr(),
                                 loss.data_ptr(), work.data_ptr(), _stream_ptr(x.device)), "gt_mlp_gradient")
    return y, g, loss


def mlp_adam(params, grad, m1, m2, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    _check(lib().gt_mlp_adam(params.data_ptr(), grad.data_ptr(), m1.data_ptr(), m2.data_ptr(), step, lr, beta1,
                             beta2, eps, _stream_ptr(params.device)), "gt_mlp_adam")


# ---- random-access microbenchmark (Fig. 3; the per-access times of Eq. 2 / Eq. 3)
ACCESS_READ, ACCESS_WRITE, ACCESS_ATOMIC, ACCESS_INDEX = range(4)
MEMORY_GLOBAL, MEMORY_LDS = range(2)
THREADS_PER_BLOCK = 256


def random_access(buf, words, kind, memory, seed, per_thread, blocks, sink=None):
    """Enqueue one microbenchmark launch on the current stream.  ``buf`` is a
    32-bit tensor of at least ``words`` (GLOBAL) or ``blocks * words`` (LDS)
    elements; ``sink`` None or a 32-bit tensor of ``blocks * 256`` elements."""
    need = words * (blocks if memory == MEMORY_LDS else 1)
    if buf.element_size() != 4 or buf.numel() < need:
        raise ValueError(f"buf needs {need} 32-bit words")
    if sink is not None and (sink.element_size() != 4 or sink.numel() < blocks * THREADS_PER_BLOCK):
        raise ValueError(f"sink needs {blocks * THREADS_PER_BLOCK} 32-bit words")
    _check(lib().gt_random_access(buf.data_ptr(), words, kind, memory, seed & 0xFFFFFFFF, per_thread, blocks,
                                  sink.data_ptr() if sink is not None else None, _stream_ptr(buf.device)),
           "gt_random_access")
