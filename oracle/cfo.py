"""ctypes binding of the FP64 CPU oracle (oracle/libcfo.so).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only users.  It imports nothing from the GPU package;
it takes scene dictionaries (plain numpy arrays) as produced by the seeded
scene generators.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# CFO_LIB names another build of the same source (the sanitizer test's)
LIB = os.environ.get("CFO_LIB") or os.path.join(HERE, "libcfo.so")
SRC = os.path.join(HERE, "cfo.c")
HDR = os.path.join(HERE, "cfo.h")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


class _Desc(C.Structure):
    _fields_ = [
        ("nworld", C.c_int), ("nbody", C.c_int), ("ngeom", C.c_int), ("ncon_max", C.c_int),
        ("condim", C.c_int),
        ("body_parent", _ip), ("body_jnt", _ip),
        ("body_pos", _dp), ("body_quat", _dp), ("body_ipos", _dp), ("jnt_axis", _dp),
        ("body_mass", _dp), ("body_inertia", _dp),
        ("geom_type", _ip), ("geom_body", _ip),
        ("geom_size", _dp), ("geom_pos", _dp), ("geom_quat", _dp), ("geom_friction", _dp),
        ("h", C.c_double), ("gravity", C.c_double * 3), ("k_user", C.c_double),
        ("d_user", C.c_double), ("solimp", C.c_double * 5), ("margin", C.c_double),
        ("impedance", C.c_int),
        ("dof_kp", _dp), ("dof_kd", _dp),
    ]


class _Out(C.Structure):
    _fields_ = [
        ("ncon", _ip), ("overflow", _ip), ("geom", _ip), ("sub", _ip),
        ("dist", _dp), ("pos", _dp), ("frame", _dp), ("impulse", _dp),
        ("guard_phi", _dp), ("guard_frame", _dp), ("v_smooth", _dp), ("gen_impulse", _dp),
        ("trace", _dp), ("facet_gain", _dp), ("features", _dp), ("fallback", _ip),
        ("fallback_slack", _dp),
    ]


def build(force: bool = False, path: str | None = None, sanitize: bool = False) -> str:
    """Compile libcfo.so with gcc (portable -O2, no fast-math).

    sanitize: AddressSanitizer + UndefinedBehaviorSanitizer build (-O1, every
    finding fatal), for the test that runs the oracle's pins on it."""
    out = path or LIB
    if (not force and os.path.exists(out)
            and os.path.getmtime(out) >= max(os.path.getmtime(SRC), os.path.getmtime(HDR))):
        return out
    tmp = out + ".tmp"
    opt = (["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
            "-fno-sanitize-recover=all"] if sanitize else ["-O2"])
    subprocess.check_call(["gcc", "-std=c99", *opt, "-fno-fast-math", "-Wall", "-fPIC",
                           "-shared", "-o", tmp, SRC, "-lm"])
    os.replace(tmp, out)
    return out


_lib = None
_lock = threading.Lock()


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB):
                build()
            L = C.CDLL(LIB)
            L.cfo_create.argtypes = [C.POINTER(_Desc), C.POINTER(C.c_void_p), C.c_char_p, C.c_int]
            L.cfo_create.restype = C.c_int
            L.cfo_destroy.argtypes = [C.c_void_p]
            L.cfo_dims.argtypes = [C.c_void_p, _ip, _ip, _ip]
            L.cfo_step.argtypes = [C.c_void_p, C.c_int, C.c_int, _dp, _dp, _dp, _dp, _dp,
                                   C.POINTER(_Out)]
            L.cfo_step.restype = C.c_int
            L.cfo_body_frames.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _dp]
            L.cfo_body_jacobian.argtypes = [C.c_void_p, C.c_int, _dp, C.c_int, _dp]
            L.cfo_mass_matrix.argtypes = [C.c_void_p, C.c_int, _dp, _dp]
            L.cfo_bias.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _dp]
            L.cfo_impedance_ratio.argtypes = [C.c_void_p, C.c_double]
            L.cfo_impedance_ratio.restype = C.c_double
            L.cfo_gamma.argtypes = [C.c_void_p, C.c_double]
            L.cfo_gamma.restype = C.c_double
            L.cfo_set_learned.argtypes = [C.c_void_p, _dp, C.c_double]
            L.cfo_set_learned.restype = C.c_int
            _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def _i(a):
    return a.ctypes.data_as(_ip) if a is not None else None


class OracleError(RuntimeError):
    pass


class Oracle:
    """FP64 oracle model built from a scene dictionary."""

    def __init__(self, scene):
        L = lib()
        self.scene = scene
        nw, nb, ng = scene["nworld"], scene["nbody"], scene["ngeom"]
        keep = {}

        def arr(key, dtype):
            a = np.ascontiguousarray(scene[key], dtype=dtype)
            keep[key] = a
            return a

        d = _Desc()
        d.nworld, d.nbody, d.ngeom = nw, nb, ng
        d.ncon_max, d.condim = int(scene["ncon_max"]), int(scene["condim"])
        d.body_parent = _i(arr("body_parent", np.int32))
        d.body_jnt = _i(arr("body_jnt", np.int32))
        for k in ("body_pos", "body_quat", "body_ipos", "jnt_axis", "body_mass", "body_inertia",
                  "geom_size", "geom_pos", "geom_quat", "geom_friction"):
            setattr(d, k, _d(arr(k, np.float64)))
        d.geom_type = _i(arr("geom_type", np.int32))
        d.geom_body = _i(arr("geom_body", np.int32))
        d.h = float(scene["h"])
        d.gravity[:] = [float(x) for x in scene["gravity"]]
        d.k_user, d.d_user = float(scene["k_user"]), float(scene["d_user"])
        d.solimp[:] = [float(x) for x in scene["solimp"]]
        d.margin = float(scene["margin"])
        d.impedance = int(scene.get("impedance", 0))
        if scene.get("dof_kp") is not None or scene.get("dof_kd") is not None:
            nv = sum({0: 6, 1: 1, 2: 1}[int(t)] for t in scene["body_jnt"])
            for key in ("dof_kp", "dof_kd"):
                val = scene.get(key)
                a = np.zeros(nv) if val is None else np.ascontiguousarray(val, dtype=np.float64)
                keep[key] = a
                setattr(d, key, _d(a))
        self._keep = keep
        h = C.c_void_p()
        err = C.create_string_buffer(256)
        rc = L.cfo_create(C.byref(d), C.byref(h), err, 256)
        if rc != 0:
            raise OracleError(f"cfo_create failed ({rc}): {err.value.decode()}")
        self._h = h
        nq, nv, nf = C.c_int(), C.c_int(), C.c_int()
        L.cfo_dims(h, C.byref(nq), C.byref(nv), C.byref(nf))
        self.nq, self.nv, self.nf = nq.value, nv.value, nf.value
        self.nworld, self.nbody, self.ngeom = nw, nb, ng
        self.ncon_max = int(scene["ncon_max"])

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().cfo_destroy(h)
            self._h = None

    # ---------------------------------------------------------------- step
    def step(self, q, v, tau=None, worlds=None, outputs=True, learned=None):
        """One step of every world (or of the range/list `worlds`).

        Returns (q_out, v_out, out) with float64 arrays; out holds the contact
        list, facet impulses, guards and intermediates when outputs=True.
        learned = (params, margin) or (params, margin, operands): the learned
        impedance gains of the network `params` (oracle/mlp.py layout) with the
        fallback margin (m): a plain step of the same state exports each
        contact's features, the network maps them to its outputs (in float64,
        or with operands="bf16" at a bf16 matrix unit's operand precision), and
        the step is taken again with them; out["learned_y"] holds the outputs.
        """
        if learned is None:
            return self._step(q, v, tau, worlds, outputs)
        from oracle import mlp
        params, margin = learned[0], learned[1]
        operands = learned[2] if len(learned) > 2 else None
        _, _, o1 = self._step(q, v, tau, worlds, True)
        y, _ = mlp.forward(params, o1["features"].reshape(-1, mlp.NIN), operands=operands)
        y = np.ascontiguousarray(y.reshape(self.nworld, self.ncon_max, mlp.NOUT))
        L = lib()
        if L.cfo_set_learned(self._h, _d(y), float(margin)) != 0:
            raise OracleError("cfo_set_learned failed (heuristic impedance only, margin >= 0)")
        try:
            qo, vo, out = self._step(q, v, tau, worlds, True)
        finally:
            L.cfo_set_learned(self._h, None, 0.0)
        out["learned_y"] = y
        return qo, vo, out

    def _step(self, q, v, tau, worlds, outputs):
        nw, nq, nv = self.nworld, self.nq, self.nv
        q = np.ascontiguousarray(q, np.float64).reshape(nw, nq)
        v = np.ascontiguousarray(v, np.float64).reshape(nw, nv)
        tau_a = None if tau is None else np.ascontiguousarray(tau, np.float64).reshape(nw, nv)
        qo, vo = q.copy(), v.copy()
        out, o = None, None
        if outputs:
            cm, nf = self.ncon_max, self.nf
            out = dict(
                ncon=np.zeros(nw, np.int32), overflow=np.zeros(nw, np.int32),
                geom=np.full((nw, cm, 2), -1, np.int32), sub=np.full((nw, cm), -1, np.int32),
                dist=np.zeros((nw, cm)), pos=np.zeros((nw, cm, 3)), frame=np.zeros((nw, cm, 9)),
                impulse=np.zeros((nw, cm, nf)), guard_phi=np.full(nw, np.inf),
                guard_frame=np.full(nw, np.inf), v_smooth=np.zeros((nw, nv)),
                gen_impulse=np.zeros((nw, nv)), trace=np.zeros((nw, self.nbody)),
                facet_gain=np.zeros((nw, cm, nf)), features=np.zeros((nw, cm, 8)),
                fallback=np.full((nw, cm), -1, np.int32), fallback_slack=np.zeros((nw, cm, 2)))
            o = _Out()
            for k in ("ncon", "overflow", "geom", "sub", "fallback"):
                setattr(o, k, _i(out[k]))
            for k in ("dist", "pos", "frame", "impulse", "guard_phi", "guard_frame", "v_smooth",
                      "gen_impulse", "trace", "facet_gain", "features", "fallback_slack"):
                setattr(o, k, _d(out[k]))
        if worlds is None:
            ranges = [(0, nw)]
        else:
            ranges = [(int(w), int(w) + 1) for w in worlds]
        L = lib()
        for w0, w1 in ranges:
            rc = L.cfo_step(self._h, w0, w1, _d(q), _d(v), _d(tau_a), _d(qo), _d(vo),
                            C.byref(o) if o is not None else None)
            if rc != 0:
                raise OracleError(f"cfo_step failed ({rc}) in worlds [{w0},{w1})")
        return qo, vo, out

    def step_threads(self, q, v, nthreads, tau=None):
        """One step of all worlds with worlds split statically over nthreads threads
        (the C call releases the GIL).  No outputs beyond the state."""
        nw, nq, nv = self.nworld, self.nq, self.nv
        q = np.ascontiguousarray(q, np.float64).reshape(nw, nq)
        v = np.ascontiguousarray(v, np.float64).reshape(nw, nv)
        tau_a = None if tau is None else np.ascontiguousarray(tau, np.float64).reshape(nw, nv)
        qo, vo = q.copy(), v.copy()
        L = lib()
        bounds = np.linspace(0, nw, nthreads + 1).astype(int)
        errs = []

        def run(w0, w1):
            if w1 > w0:
                rc = L.cfo_step(self._h, int(w0), int(w1), _d(q), _d(v), _d(tau_a), _d(qo),
                                _d(vo), None)
                if rc != 0:
                    errs.append(rc)

        th = [threading.Thread(target=run, args=(bounds[i], bounds[i + 1]))
              for i in range(nthreads)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        if errs:
            raise OracleError(f"cfo_step failed {errs}")
        return qo, vo

    def rollout(self, steps, q0=None, v0=None, tau=None, record=False):
        q = np.asarray(self.scene["q0"] if q0 is None else q0, np.float64)
        v = np.asarray(self.scene["v0"] if v0 is None else v0, np.float64)
        traj = [(q, v)] if record else None
        outs = []
        for _ in range(steps):
            q, v, out = self.step(q, v, tau, outputs=record)
            if record:
                traj.append((q, v))
                outs.append(out)
        return (q, v, traj, outs) if record else (q, v)

    # ------------------------------------------------------- building blocks
    def frames(self, w, q):
        com = np.zeros((self.nbody, 3))
        rot = np.zeros((self.nbody, 9))
        q = np.ascontiguousarray(q, np.float64)
        lib().cfo_body_frames(self._h, w, _d(q), _d(com), _d(rot))
        return com, rot.reshape(self.nbody, 3, 3)

    def jacobian(self, w, q, body):
        J = np.zeros((6, self.nv))
        q = np.ascontiguousarray(q, np.float64)
        lib().cfo_body_jacobian(self._h, w, _d(q), body, _d(J))
        return J

    def mass_matrix(self, w, q):
        M = np.zeros((self.nv, self.nv))
        q = np.ascontiguousarray(q, np.float64)
        lib().cfo_mass_matrix(self._h, w, _d(q), _d(M))
        return M

    def bias(self, w, q, v):
        c = np.zeros(self.nv)
        q = np.ascontiguousarray(q, np.float64)
        v = np.ascontiguousarray(v, np.float64)
        lib().cfo_bias(self._h, w, _d(q), _d(v), _d(c))
        return c

    def impedance_ratio(self, phi):
        return lib().cfo_impedance_ratio(self._h, float(phi))

    def gamma(self, x):
        return lib().cfo_gamma(self._h, float(x))
