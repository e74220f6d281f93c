"""Thin ctypes binding of libcfsim.so (include/cfsim.h).

Argument marshalling only: every stage of the step runs in the library's HIP
kernels.  PyTorch supplies device memory and the stream.  There is no CPU
fallback: if the library is missing, loading fails with an error.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "_lib", "libcfsim.so")

CF_OK, CF_W_PAIRS_SKIPPED = 0, 1
CF_E_INVALID_ARG, CF_E_DEVICE, CF_E_NOMEM, CF_E_UNSUPPORTED = -1, -2, -3, -4
_NAMES = {0: "CF_OK", 1: "CF_W_PAIRS_SKIPPED", -1: "CF_E_INVALID_ARG", -2: "CF_E_DEVICE",
          -3: "CF_E_NOMEM", -4: "CF_E_UNSUPPORTED"}

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_fp = C.c_void_p


class ModelDesc(C.Structure):
    _fields_ = [
        ("nworld", C.c_int32), ("nbody", C.c_int32), ("ngeom", C.c_int32),
        ("ncon_max", C.c_int32), ("condim", C.c_int32),
        ("body_parent", _ip), ("body_jnt", _ip),
        ("body_pos", _dp), ("body_quat", _dp), ("body_ipos", _dp), ("jnt_axis", _dp),
        ("body_mass", _dp), ("body_inertia", _dp),
        ("geom_type", _ip), ("geom_body", _ip),
        ("geom_size", _dp), ("geom_pos", _dp), ("geom_quat", _dp), ("geom_friction", _dp),
        ("h", C.c_double), ("gravity", C.c_double * 3), ("k_user", C.c_double),
        ("d_user", C.c_double), ("solimp", C.c_double * 5), ("margin", C.c_double),
    ]


class Contacts(C.Structure):
    _fields_ = [("ncon", C.c_void_p), ("overflow", C.c_void_p), ("geom", C.c_void_p),
                ("sub", C.c_void_p), ("dist", C.c_void_p), ("pos", C.c_void_p),
                ("frame", C.c_void_p), ("impulse", C.c_void_p), ("features", C.c_void_p),
                ("target", C.c_void_p), ("fallback", C.c_void_p)]


class CFError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None

# Every symbol declared in include/cfsim.h, with its ctypes signature.
SIGNATURES = {
    "cf_model_create": ([C.POINTER(ModelDesc), C.POINTER(C.c_void_p)], C.c_int32),
    "cf_model_destroy": ([C.c_void_p], None),
    "cf_model_dims": ([C.c_void_p, _ip, _ip, _ip], C.c_int32),
    "cf_step": ([C.c_void_p, C.c_void_p, _fp, _fp, _fp, _fp, _fp, C.POINTER(Contacts)], C.c_int32),
    "cf_rollout": ([C.c_void_p, C.c_void_p, C.c_int32, _fp, _fp, _fp, _fp, _fp, _fp, _fp], C.c_int32),
    "cf_step_backward": ([C.c_void_p, C.c_void_p, _fp, _fp, _fp, _fp, _fp, _fp, _fp, _fp], C.c_int32),
    "cf_model_set_launch": ([C.c_void_p, C.c_int32, C.c_int32, C.c_int32], C.c_int32),
    "cf_model_set_impedance": ([C.c_void_p, C.c_int32], C.c_int32),
    "cf_model_set_actuators": ([C.c_void_p, C.POINTER(C.c_float), C.POINTER(C.c_float)], C.c_int32),
    "cf_model_set_learned_impedance": ([C.c_void_p, _fp, C.c_float], C.c_int32),
    "cf_model_get_launch": ([C.c_void_p, _ip, _ip, _ip, _ip], C.c_int32),
    "cf_model_autotune": ([C.c_void_p, C.c_void_p, _fp, _fp, C.c_int32, C.POINTER(C.c_float),
                           C.POINTER(C.c_float)], C.c_int32),
    "cf_model_step_kernels": ([C.c_void_p, _ip], C.c_int32),
    "cf_model_set_profiling": ([C.c_void_p, C.c_int32], C.c_int32),
    "cf_model_kernel_times": ([C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double),
                               C.POINTER(C.c_int64)], C.c_int32),
    "cf_model_time_kernels": ([C.c_void_p, C.c_void_p, _fp, _fp, _fp, _fp, C.c_int32, C.POINTER(C.c_float),
                               C.POINTER(C.c_float)], C.c_int32),
    "cf_mlp_nparam": ([], C.c_int32),
    "cf_mlp_forward": ([C.c_void_p, _fp, _fp, C.c_int32, _fp], C.c_int32),
    "cf_mlp_work_floats": ([C.c_int32], C.c_int64),
    "cf_mlp_gradient": ([C.c_void_p, _fp, _fp, _fp, C.c_int32, C.c_int32, _fp, C.c_int64, _fp, _fp], C.c_int32),
    "cf_mlp_gradient_noalloc": ([C.c_void_p, _fp, _fp, _fp, C.c_int32, C.c_int32, _fp, _fp], C.c_int32),
    "cf_mlp_adam": ([C.c_void_p, _fp, _fp, _fp, _fp, C.c_int32, C.c_float], C.c_int32),
    "cf_last_error": ([], C.c_char_p),
}


def load(path: str = LIB_PATH):
    """Load libcfsim.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # torch first: the library then binds to the HIP runtime torch loaded
        # (a second runtime loaded ahead of torch's leaves one of them without
        # the device)
        import torch  # noqa: F401
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with paper_2603_12185_amd.build.build()")
        L = C.CDLL(path)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def last_error() -> str:
    return load().cf_last_error().decode()


def _check(st):
    if st < 0:
        raise CFError(st, last_error())
    return st


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def make_desc(scene):
    """ModelDesc from a scene dictionary; returns (desc, keepalive)."""
    keep = {}

    def arr(key, dtype, shape_check=None):
        a = np.ascontiguousarray(scene[key], dtype=dtype)
        keep[key] = a
        return a

    d = ModelDesc()
    d.nworld, d.nbody, d.ngeom = int(scene["nworld"]), int(scene["nbody"]), int(scene["ngeom"])
    d.ncon_max, d.condim = int(scene["ncon_max"]), int(scene["condim"])
    d.body_parent = arr("body_parent", np.int32).ctypes.data_as(_ip)
    d.body_jnt = arr("body_jnt", np.int32).ctypes.data_as(_ip)
    d.geom_type = arr("geom_type", np.int32).ctypes.data_as(_ip)
    d.geom_body = arr("geom_body", np.int32).ctypes.data_as(_ip)
    for k in ("body_pos", "body_quat", "body_ipos", "jnt_axis", "body_mass", "body_inertia",
              "geom_size", "geom_pos", "geom_quat", "geom_friction"):
        setattr(d, k, arr(k, np.float64).ctypes.data_as(_dp))
    d.h = float(scene["h"])
    d.gravity[:] = [float(x) for x in scene["gravity"]]
    d.k_user, d.d_user = float(scene["k_user"]), float(scene["d_user"])
    d.solimp[:] = [float(x) for x in scene["solimp"]]
    d.margin = float(scene["margin"])
    return d, keep


class Model:
    """A cf_model on the current HIP device."""

    def __init__(self, scene):
        import torch
        # torch's HIP context first: the library's own first HIP call would
        # otherwise leave torch unable to initialise the device
        if not torch.cuda.is_available():
            raise RuntimeError("cfsim.Model needs a HIP device")
        L = load()
        d, keep = make_desc(scene)
        h = C.c_void_p()
        st = _check(L.cf_model_create(C.byref(d), C.byref(h)))
        self.warning = last_error() if st == CF_W_PAIRS_SKIPPED else ""
        self._h = h
        nq, nv, nf = C.c_int32(), C.c_int32(), C.c_int32()
        _check(L.cf_model_dims(h, C.byref(nq), C.byref(nv), C.byref(nf)))
        self.nq, self.nv, self.nfacet = nq.value, nv.value, nf.value
        self.nworld = int(scene["nworld"])
        self.ncon_max = int(scene["ncon_max"])
        self.nbody, self.ngeom = int(scene["nbody"]), int(scene["ngeom"])
        if int(scene.get("impedance", 0)):
            self.set_impedance(int(scene["impedance"]))
        if scene.get("dof_kp") is not None or scene.get("dof_kd") is not None:
            self.set_actuators(scene.get("dof_kp"), scene.get("dof_kd"))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().cf_model_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ buffers
    def _check_state(self, t, cols, name):
        import torch
        if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
        if t.numel() != self.nworld * cols:
            raise ValueError(f"{name} must hold nworld*{cols} = {self.nworld * cols} values")

    def alloc_contacts(self, device="cuda", training=False):
        """Device tensors for every contact output of a step (with the
        learned-gain training data when `training`)."""
        import torch
        nw, cm, nf = self.nworld, self.ncon_max, self.nfacet
        i32, f32 = torch.int32, torch.float32
        return dict(
            ncon=torch.zeros(nw, dtype=i32, device=device),
            overflow=torch.zeros(nw, dtype=i32, device=device),
            geom=torch.full((nw, cm, 2), -1, dtype=i32, device=device),
            sub=torch.full((nw, cm), -1, dtype=i32, device=device),
            dist=torch.zeros((nw, cm), dtype=f32, device=device),
            pos=torch.zeros((nw, cm, 3), dtype=f32, device=device),
            frame=torch.zeros((nw, cm, 9), dtype=f32, device=device),
            impulse=torch.zeros((nw, cm, nf), dtype=f32, device=device),
            **({} if not training else dict(features=torch.zeros((nw, cm, 8), dtype=f32, device=device),
                                            target=torch.zeros((nw, cm, 16), dtype=f32, device=device))))

    # ------------------------------------------------------------ compute
    def step(self, q, v, tau=None, q_out=None, v_out=None, contacts=None, stream=None):
        """One step of every world on `stream` (default: torch's current stream)."""
        import torch
        self._check_state(q, self.nq, "q")
        self._check_state(v, self.nv, "v")
        if tau is not None:
            self._check_state(tau, self.nv, "tau")
        q_out = torch.empty_like(q) if q_out is None else q_out
        v_out = torch.empty_like(v) if v_out is None else v_out
        self._check_state(q_out, self.nq, "q_out")
        self._check_state(v_out, self.nv, "v_out")
        c = None
        if contacts is not None:
            c = Contacts(*[_ptr(contacts.get(k)) for k, _ in Contacts._fields_])
        s = torch.cuda.current_stream() if stream is None else stream
        _check(load().cf_step(self._h, C.c_void_p(s.cuda_stream), _ptr(q), _ptr(v), _ptr(tau),
                              _ptr(q_out), _ptr(v_out), C.byref(c) if c is not None else None))
        return q_out, v_out

    def step_backward(self, q, v, tau, gq_out, gv_out, gq=None, gv=None, gtau=None, stream=None):
        """Adjoint of step(q, v, tau): returns (gq, gv, gtau) = the gradients of
        <gq_out, q+> + <gv_out, v+> with respect to q, v and tau (contact set
        and facet activity held at the forward point)."""
        import torch
        self._check_state(q, self.nq, "q")
        self._check_state(v, self.nv, "v")
        if tau is not None:
            self._check_state(tau, self.nv, "tau")
        if gq_out is not None:
            self._check_state(gq_out, self.nq, "gq_out")
        if gv_out is not None:
            self._check_state(gv_out, self.nv, "gv_out")
        gq = torch.empty_like(q) if gq is None else gq
        gv = torch.empty_like(v) if gv is None else gv
        gtau = torch.empty_like(v) if gtau is None else gtau
        self._check_state(gq, self.nq, "gq")
        self._check_state(gv, self.nv, "gv")
        self._check_state(gtau, self.nv, "gtau")
        s = torch.cuda.current_stream() if stream is None else stream
        _check(load().cf_step_backward(self._h, C.c_void_p(s.cuda_stream), _ptr(q), _ptr(v), _ptr(tau),
                                       _ptr(gq_out), _ptr(gv_out), _ptr(gq), _ptr(gv), _ptr(gtau)))
        return gq, gv, gtau

    def rollout(self, T, q0, v0, tau_seq=None, q_traj=None, v_traj=None, ncon_traj=None,
                stream=None, overflow_traj=None):
        """T steps; returns trajectories [T+1][nworld][nq|nv] (ncon_traj and
        overflow_traj, int32 [T][nworld], receive per-step contact counts kept
        and dropped beyond ncon_max when given)."""
        import torch
        self._check_state(q0, self.nq, "q0")
        self._check_state(v0, self.nv, "v0")
        if q_traj is None:
            q_traj = torch.empty((T + 1, self.nworld, self.nq), dtype=torch.float32, device=q0.device)
        if v_traj is None:
            v_traj = torch.empty((T + 1, self.nworld, self.nv), dtype=torch.float32, device=v0.device)
        if tau_seq is not None and (tau_seq.numel() != T * self.nworld * self.nv
                                    or not tau_seq.is_contiguous()):
            raise ValueError("tau_seq must be contiguous [T][nworld][nv]")
        s = torch.cuda.current_stream() if stream is None else stream
        for name, t in (("ncon_traj", ncon_traj), ("overflow_traj", overflow_traj)):
            if t is not None and (t.dtype != torch.int32 or t.numel() < T * self.nworld
                                  or not t.is_contiguous()):
                raise ValueError(f"{name} must be contiguous int32 [T][nworld]")
        _check(load().cf_rollout(self._h, C.c_void_p(s.cuda_stream), int(T), _ptr(q0), _ptr(v0),
                                 _ptr(tau_seq), _ptr(q_traj), _ptr(v_traj), _ptr(ncon_traj),
                                 _ptr(overflow_traj)))
        return q_traj, v_traj

    # ------------------------------------------------------------ launch shape
    def set_learned_impedance(self, net, margin=0.0):
        """Scale the heuristic gains by the network `net` (an ImpedanceNet, or
        None to switch it off) with the given fallback margin in metres."""
        self._net = net  # the library reads the parameters at every step
        _check(load().cf_model_set_learned_impedance(self._h, None if net is None else _ptr(net.params),
                                                     float(margin)))

    def set_actuators(self, kp, kd):
        """Position actuators: per-dof gains (host sequences of nv values, None =
        zeros; both None removes them).  The step input of an actuated dof is
        then its target position."""
        def arr(x):
            if x is None:
                return None
            a = np.ascontiguousarray(x, dtype=np.float32)
            if a.shape != (self.nv,):
                raise ValueError(f"actuator gains must have nv = {self.nv} entries")
            return a
        a, b = arr(kp), arr(kd)
        fp = C.POINTER(C.c_float)
        _check(load().cf_model_set_actuators(self._h, None if a is None else a.ctypes.data_as(fp),
                                             None if b is None else b.ctypes.data_as(fp)))

    def set_impedance(self, mode):
        """0: heuristic impedance (default); 1: exact diagonal impedance per facet."""
        _check(load().cf_model_set_impedance(self._h, int(mode)))

    def set_launch(self, collide_block, resolve_block, rollout_block=None):
        if rollout_block is None:
            rollout_block = self.get_launch()[2]
        _check(load().cf_model_set_launch(self._h, int(collide_block), int(resolve_block),
                                          int(rollout_block)))

    def get_launch(self):
        """(collide_block, resolve_block, rollout_block, rollout_uses_persistent_kernel)."""
        a, b, c, d = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(load().cf_model_get_launch(self._h, C.byref(a), C.byref(b), C.byref(c), C.byref(d)))
        return a.value, b.value, c.value, bool(d.value)

    def step_kernels(self):
        """1 when cf_step runs the narrow phase and the resolution in one kernel, else 2."""
        n = C.c_int32()
        _check(load().cf_model_step_kernels(self._h, C.byref(n)))
        return n.value

    def autotune(self, q, v, steps=20, stream=None):
        """Pick the fastest workgroup sizes on state (q, v); returns (us/step of
        cf_step, us/step of cf_rollout or -1)."""
        import torch
        self._check_state(q, self.nq, "q")
        self._check_state(v, self.nv, "v")
        s = torch.cuda.current_stream() if stream is None else stream
        a, b = C.c_float(), C.c_float()
        _check(load().cf_model_autotune(self._h, C.c_void_p(s.cuda_stream), _ptr(q), _ptr(v),
                                        int(steps), C.byref(a), C.byref(b)))
        return a.value, b.value

    # ------------------------------------------------------------ timing
    def set_profiling(self, on: bool):
        _check(load().cf_model_set_profiling(self._h, 1 if on else 0))

    def time_kernels(self, q, v, q_out, v_out, reps=200, stream=None):
        """Average microseconds per launch of the collision and the resolution
        kernel, each launched `reps` times back to back from (q, v)."""
        import torch
        for t, n, name in ((q, self.nq, "q"), (v, self.nv, "v"), (q_out, self.nq, "q_out"),
                           (v_out, self.nv, "v_out")):
            self._check_state(t, n, name)
        s = torch.cuda.current_stream() if stream is None else stream
        a, b = C.c_float(), C.c_float()
        _check(load().cf_model_time_kernels(self._h, C.c_void_p(s.cuda_stream), _ptr(q), _ptr(v), _ptr(q_out),
                                            _ptr(v_out), int(reps), C.byref(a), C.byref(b)))
        return a.value, b.value

    def kernel_times(self):
        """(ms_collide, ms_resolve, steps) summed since the last call."""
        a, b, n = C.c_double(), C.c_double(), C.c_int64()
        _check(load().cf_model_kernel_times(self._h, C.byref(a), C.byref(b), C.byref(n)))
        return a.value, b.value, n.value


# ---------------------------------------------------------------- learned impedance network
class ImpedanceNet:
    """Device-side parameters of the learned impedance network and its training
    state (Adam moments); every computation runs in the library's kernels."""

    def __init__(self, params):
        import torch
        L = load()
        self.nparam = int(L.cf_mlp_nparam())
        p = torch.as_tensor(params, dtype=torch.float32).reshape(-1)
        if p.numel() != self.nparam:
            raise ValueError(f"expected {self.nparam} parameters")
        self.params = p.cuda().contiguous()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0
        self._work = None

    @staticmethod
    def _check(t, cols, name):
        import torch
        if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or t.dim() != 2 \
                or t.shape[1] != cols:
            raise ValueError(f"{name} must be a contiguous float32 CUDA tensor [n][{cols}]")

    def forward(self, feats, out=None, stream=None):
        import torch
        self._check(feats, 8, "feats")
        n = feats.shape[0]
        out = torch.empty((n, 16), dtype=torch.float32, device=feats.device) if out is None else out
        s = torch.cuda.current_stream() if stream is None else stream
        _check(load().cf_mlp_forward(C.c_void_p(s.cuda_stream), _ptr(self.params), _ptr(feats), n, _ptr(out)))
        return out

    def gradient(self, feats, targets, nout, stream=None):
        """(grad [nparam], loss) of the mean squared error; both device tensors."""
        import torch
        self._check(feats, 8, "feats")
        self._check(targets, 16, "targets")
        n = feats.shape[0]
        need = int(load().cf_mlp_work_floats(n))
        if self._work is None or self._work.numel() < need:
            self._work = torch.empty(need, dtype=torch.float32, device=feats.device)
        grad = torch.empty_like(self.params)
        loss = torch.empty(1, dtype=torch.float32, device=feats.device)
        s = torch.cuda.current_stream() if stream is None else stream
        _check(load().cf_mlp_gradient(C.c_void_p(s.cuda_stream), _ptr(self.params), _ptr(feats), _ptr(targets), n,
                                      int(nout), _ptr(self._work), self._work.numel(), _ptr(grad), _ptr(loss)))
        return grad, loss

    def gradient_noalloc(self, feats, targets, nout, grad, loss, stream=None):
        """gradient() through the entry point that allocates nothing: the
        caller passes the outputs grad [nparam] and loss [1]."""
        import torch
        self._check(feats, 8, "feats")
        self._check(targets, 16, "targets")
        for t, k, name in ((grad, self.nparam, "grad"), (loss, 1, "loss")):
            if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or t.numel() != k:
                raise ValueError(f"{name} must be a contiguous float32 CUDA tensor of {k} values")
        s = torch.cuda.current_stream() if stream is None else stream
        _check(load().cf_mlp_gradient_noalloc(C.c_void_p(s.cuda_stream), _ptr(self.params), _ptr(feats),
                                              _ptr(targets), feats.shape[0], int(nout), _ptr(grad), _ptr(loss)))
        return grad, loss

    def train_step(self, feats, targets, nout, lr, stream=None):
        import torch
        grad, loss = self.gradient(feats, targets, nout, stream)
        self.step += 1
        s = torch.cuda.current_stream() if stream is None else stream
        _check(load().cf_mlp_adam(C.c_void_p(s.cuda_stream), _ptr(self.params), _ptr(self.m), _ptr(self.v),
                                  _ptr(grad), self.step, float(lr)))
        return loss
