"""ctypes front end of the CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It loads oracle/liboracle.so (built by build_oracle.py)
and returns numpy copies of everything it hands out.
"""
import ctypes as C
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

ARITH_INT32 = 0
ARITH_F64 = 1
W_PLAIN = 0
W_COMPRESSED = 1
W_DEV8 = 2


class _Cfg(C.Structure):
    _fields_ = [
        ("seed", C.c_uint64),
        ("scale", C.c_double),
        ("indegree_mode", C.c_int),
        ("count_rule", C.c_int),
        ("rows_are_sources", C.c_int),
        ("g", C.c_double),
        ("bg_rate_hz", C.c_double),
        ("psp_ext_mv", C.c_double),
        ("bg_const_T", C.c_int),
        ("weight_mode", C.c_int),
        ("conn", C.POINTER(C.c_double)),
    ]


class _Consts(C.Structure):
    _fields_ = [
        ("w_f", C.c_double), ("p11", C.c_double), ("p22", C.c_double), ("p21", C.c_double),
        ("p11f", C.c_float), ("p22f", C.c_float), ("p21f", C.c_float),
        ("w_ext", C.c_double), ("w_ext_q", C.c_int32),
    ]


class _Counters(C.Structure):
    _fields_ = [("spikes", C.c_uint64), ("events", C.c_uint64), ("poisson", C.c_uint64),
                ("consumed", C.c_int64), ("injected", C.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from oracle import build_oracle
            build_oracle.build()
        _lib = C.CDLL(LIB_PATH)
        L = _lib
        vp = C.c_void_p
        L.orc_config_default.argtypes = [C.POINTER(_Cfg)]
        L.orc_constants.argtypes = [C.POINTER(_Cfg), C.POINTER(_Consts)]
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                        C.POINTER(C.c_uint32)]
        L.orc_poisson_table.argtypes = [C.c_double, C.POINTER(C.c_uint32), C.c_int,
                                        C.POINTER(C.c_int)]
        L.orc_build.argtypes = [C.POINTER(_Cfg), C.POINTER(vp)]
        L.orc_net_free.argtypes = [vp]
        L.orc_pair_counts.argtypes = [C.POINTER(_Cfg), C.POINTER(C.c_uint64)]
        L.orc_net_n.argtypes = [vp]
        L.orc_net_n.restype = C.c_uint32
        L.orc_net_nsyn.argtypes = [vp]
        L.orc_net_nsyn.restype = C.c_uint64
        L.orc_net_pop_offsets.argtypes = [vp, C.POINTER(C.c_uint32)]
        L.orc_net_pair_count.argtypes = [vp, C.c_int, C.c_int]
        L.orc_net_pair_count.restype = C.c_uint64
        for name, rt in [("orc_net_row_ptr", C.POINTER(C.c_uint64)),
                         ("orc_net_post", C.POINTER(C.c_uint32)),
                         ("orc_net_delay", C.POINTER(C.c_uint8)),
                         ("orc_net_weight", C.POINTER(C.c_double)),
                         ("orc_net_weight_q", C.POINTER(C.c_int32)),
                         ("orc_net_u0", C.POINTER(C.c_float)),
                         ("orc_net_u0_f64", C.POINTER(C.c_double))]:
            getattr(L, name).argtypes = [vp]
            getattr(L, name).restype = rt
        L.orc_net_poisson.argtypes = [vp, C.c_int, C.POINTER(C.POINTER(C.c_uint32)),
                                      C.POINTER(C.c_int)]
        L.orc_sim_new.argtypes = [vp, C.c_int, C.POINTER(vp)]
        L.orc_sim_free.argtypes = [vp]
        L.orc_sim_set_probes.argtypes = [vp, C.POINTER(C.c_uint32), C.c_uint32]
        L.orc_sim_record_inputs.argtypes = [vp, C.c_int]
        L.orc_sim_run.argtypes = [vp, C.c_uint64]
        L.orc_sim_run_threads.argtypes = [vp, C.c_uint64, C.c_int]
        L.orc_sim_t.argtypes = [vp]
        L.orc_sim_t.restype = C.c_uint64
        L.orc_sim_counters.argtypes = [vp, C.POINTER(_Counters)]
        for name in ["orc_sim_nspikes", "orc_sim_probe_steps", "orc_sim_rec_steps"]:
            getattr(L, name).argtypes = [vp]
            getattr(L, name).restype = C.c_uint64
        for name, rt in [("orc_sim_spike_steps", C.POINTER(C.c_uint32)),
                         ("orc_sim_spike_ids", C.POINTER(C.c_uint32)),
                         ("orc_sim_u", C.POINTER(C.c_float)),
                         ("orc_sim_i", C.POINTER(C.c_float)),
                         ("orc_sim_u64", C.POINTER(C.c_double)),
                         ("orc_sim_i64", C.POINTER(C.c_double)),
                         ("orc_sim_r", C.POINTER(C.c_int32)),
                         ("orc_sim_ring_q", C.POINTER(C.c_int64)),
                         ("orc_sim_ring_f64", C.POINTER(C.c_double)),
                         ("orc_sim_probe_u", C.POINTER(C.c_float)),
                         ("orc_sim_probe_i", C.POINTER(C.c_float)),
                         ("orc_sim_probe_u64", C.POINTER(C.c_double)),
                         ("orc_sim_probe_i64", C.POINTER(C.c_double)),
                         ("orc_sim_probe_r", C.POINTER(C.c_int32)),
                         ("orc_sim_rec_T", C.POINTER(C.c_int32)),
                         ("orc_sim_rec_w", C.POINTER(C.c_int64)),
                         ("orc_sim_rec_w64", C.POINTER(C.c_double))]:
            getattr(L, name).argtypes = [vp]
            getattr(L, name).restype = rt
        L.orc_single_neuron_f32.argtypes = [C.POINTER(_Consts), C.POINTER(C.c_int64), C.c_uint64,
                                            C.POINTER(C.c_float), C.POINTER(C.c_float),
                                            C.POINTER(C.c_int32)]
        L.orc_single_neuron_f64.argtypes = [C.POINTER(_Consts), C.POINTER(C.c_double), C.c_uint64,
                                            C.POINTER(C.c_double), C.POINTER(C.c_double),
                                            C.POINTER(C.c_int32)]
        L.orc_dev8_params.argtypes = [C.c_double, C.c_double, C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int32)]
        L.orc_dev8_encode.argtypes = [C.c_double, C.c_int32, C.c_int32, C.POINTER(C.c_int32)]
        L.orc_dev8_encode.restype = C.c_int32
        L.orc_net_dev8_pair.argtypes = [vp, C.c_int, C.c_int, C.POINTER(C.c_int32),
                                        C.POINTER(C.c_int32)]
        L.orc_last_error.restype = C.c_char_p
    return _lib


class OracleError(RuntimeError):
    pass


def _check(rc):
    if rc != 0:
        raise OracleError(f"oracle error {rc}: {lib().orc_last_error().decode()}")


@dataclass
class Config:
    """Mirror of orc_config; defaults are the paper's (Tables tab:params..3)."""
    seed: int = 1
    scale: float = 1.0
    indegree_mode: int = 0
    count_rule: int = 0
    rows_are_sources: int = 0
    g: float = -4.0
    bg_rate_hz: float = 8.0
    psp_ext_mv: float = 0.15
    bg_const_T: int = -1
    weight_mode: int = W_PLAIN
    conn: Optional[Sequence[float]] = None
    _keep: list = field(default_factory=list, repr=False)

    def c(self):
        cfg = _Cfg()
        cfg.seed = self.seed
        cfg.scale = self.scale
        cfg.indegree_mode = self.indegree_mode
        cfg.count_rule = self.count_rule
        cfg.rows_are_sources = self.rows_are_sources
        cfg.g = self.g
        cfg.bg_rate_hz = self.bg_rate_hz
        cfg.psp_ext_mv = self.psp_ext_mv
        cfg.bg_const_T = self.bg_const_T
        cfg.weight_mode = self.weight_mode
        if self.conn is not None:
            arr = (C.c_double * 64)(*[float(x) for x in np.asarray(self.conn).ravel()])
            self._keep = [arr]
            cfg.conn = C.cast(arr, C.POINTER(C.c_double))
        return cfg


def constants(cfg: Optional[Config] = None) -> dict:
    cfg = cfg or Config()
    k = _Consts()
    _check(lib().orc_constants(C.byref(cfg.c()), C.byref(k)))
    return {f: getattr(k, f) for f, _ in _Consts._fields_}


def _consts_struct(cfg):
    k = _Consts()
    _check(lib().orc_constants(C.byref(cfg.c()), C.byref(k)))
    return k


def philox4x32_10(ctr, key):
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def poisson_table(lam, cap=64):
    thr = (C.c_uint32 * cap)()
    n = C.c_int()
    _check(lib().orc_poisson_table(float(lam), thr, cap, C.byref(n)))
    return np.array(thr[: n.value], dtype=np.uint64)


def dev8_params(mu, sd):
    """(mq, sq) of a pair of mean mu and standard deviation sd (pA) under W_DEV8."""
    a, b = C.c_int32(), C.c_int32()
    lib().orc_dev8_params(float(mu), float(sd), C.byref(a), C.byref(b))
    return a.value, b.value


def dev8_encode(w, mq, sq):
    """(w_q, dev) of a weight w (pA) under W_DEV8."""
    d = C.c_int32()
    wq = lib().orc_dev8_encode(float(w), int(mq), int(sq), C.byref(d))
    return wq, d.value


def pair_counts(cfg: Optional[Config] = None):
    """Synapse counts [target][source] without sampling the network."""
    cfg = cfg or Config()
    out = (C.c_uint64 * 64)()
    _check(lib().orc_pair_counts(C.byref(cfg.c()), out))
    return np.array(out[:], dtype=np.int64).reshape(8, 8)


def _arr(ptr, n, dtype):
    if n == 0 or not ptr:
        return np.zeros(0, dtype=dtype)
    return np.ctypeslib.as_array(ptr, shape=(int(n),)).astype(dtype, copy=True)


class Net:
    def __init__(self, cfg: Optional[Config] = None):
        self.cfg = cfg or Config()
        h = C.c_void_p()
        _check(lib().orc_build(C.byref(self.cfg.c()), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().orc_net_free(self.h)
            self.h = None

    def __del__(self):
        self.close()

    @property
    def N(self):
        return int(lib().orc_net_n(self.h))

    @property
    def nsyn(self):
        return int(lib().orc_net_nsyn(self.h))

    def pop_offsets(self):
        o = (C.c_uint32 * 9)()
        lib().orc_net_pop_offsets(self.h, o)
        return np.array(o[:], dtype=np.int64)

    def pair_counts(self):
        L = lib()
        return np.array([[L.orc_net_pair_count(self.h, b, a) for a in range(8)] for b in range(8)],
                        dtype=np.int64)

    def csr(self):
        """(row_ptr, post, delay, w_pA, w_q) as numpy copies."""
        L = lib()
        N, S = self.N, self.nsyn
        return (_arr(L.orc_net_row_ptr(self.h), N + 1, np.uint64),
                _arr(L.orc_net_post(self.h), S, np.uint32),
                _arr(L.orc_net_delay(self.h), S, np.uint8),
                _arr(L.orc_net_weight(self.h), S, np.float64),
                _arr(L.orc_net_weight_q(self.h), S, np.int32))

    def dev8_pairs(self):
        """Mean and step (2^-8 pA) of every pair [target][source] under W_DEV8."""
        mq = np.zeros((8, 8), dtype=np.int64)
        sq = np.zeros((8, 8), dtype=np.int64)
        a, b = C.c_int32(), C.c_int32()
        for t in range(8):
            for s in range(8):
                lib().orc_net_dev8_pair(self.h, t, s, C.byref(a), C.byref(b))
                mq[t, s], sq[t, s] = a.value, b.value
        return mq, sq

    def u0(self):
        return _arr(lib().orc_net_u0(self.h), self.N, np.float32)

    def u0_f64(self):
        return _arr(lib().orc_net_u0_f64(self.h), self.N, np.float64)

    def poisson(self, p):
        t = C.POINTER(C.c_uint32)()
        n = C.c_int()
        _check(lib().orc_net_poisson(self.h, p, C.byref(t), C.byref(n)))
        return _arr(t, n.value, np.uint64)


class Sim:
    def __init__(self, net: Net, arith=ARITH_INT32, probes=None, record_inputs=False):
        self.net = net
        self.arith = arith
        h = C.c_void_p()
        _check(lib().orc_sim_new(net.h, arith, C.byref(h)))
        self.h = h
        self.nprobe = 0
        if probes is not None:
            ids = np.ascontiguousarray(probes, dtype=np.uint32)
            _check(lib().orc_sim_set_probes(self.h, ids.ctypes.data_as(C.POINTER(C.c_uint32)),
                                            len(ids)))
            self.nprobe = len(ids)
        if record_inputs:
            lib().orc_sim_record_inputs(self.h, 1)

    def close(self):
        if getattr(self, "h", None):
            lib().orc_sim_free(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def run(self, n_steps):
        _check(lib().orc_sim_run(self.h, int(n_steps)))
        return self

    def run_threads(self, n_steps, threads):
        """The same steps on `threads` host threads (INT32 arithmetic; a CPU
        baseline, equal to run() bit for bit)."""
        _check(lib().orc_sim_run_threads(self.h, int(n_steps), int(threads)))
        return self

    @property
    def t(self):
        return int(lib().orc_sim_t(self.h))

    def counters(self):
        c = _Counters()
        lib().orc_sim_counters(self.h, C.byref(c))
        return {f: int(getattr(c, f)) for f, _ in _Counters._fields_}

    def raster(self):
        L = lib()
        n = int(L.orc_sim_nspikes(self.h))
        return (_arr(L.orc_sim_spike_steps(self.h), n, np.uint32),
                _arr(L.orc_sim_spike_ids(self.h), n, np.uint32))

    def state(self):
        L = lib()
        N = self.net.N
        if self.arith == ARITH_INT32:
            u = _arr(L.orc_sim_u(self.h), N, np.float32)
            i = _arr(L.orc_sim_i(self.h), N, np.float32)
            ring = _arr(L.orc_sim_ring_q(self.h), 64 * N, np.int64).reshape(64, N)
        else:
            u = _arr(L.orc_sim_u64(self.h), N, np.float64)
            i = _arr(L.orc_sim_i64(self.h), N, np.float64)
            ring = _arr(L.orc_sim_ring_f64(self.h), 64 * N, np.float64).reshape(64, N)
        r = _arr(L.orc_sim_r(self.h), N, np.int32)
        return {"U": u, "I": i, "R": r, "W": ring, "t": self.t}

    def probes(self):
        L = lib()
        n = int(L.orc_sim_probe_steps(self.h)) * self.nprobe
        shape = (-1, self.nprobe)
        if self.arith == ARITH_INT32:
            u = _arr(L.orc_sim_probe_u(self.h), n, np.float32)
            i = _arr(L.orc_sim_probe_i(self.h), n, np.float32)
        else:
            u = _arr(L.orc_sim_probe_u64(self.h), n, np.float64)
            i = _arr(L.orc_sim_probe_i64(self.h), n, np.float64)
        r = _arr(L.orc_sim_probe_r(self.h), n, np.int32)
        return u.reshape(shape), i.reshape(shape), r.reshape(shape)

    def recorded_inputs(self):
        L = lib()
        N = self.net.N
        n = int(L.orc_sim_rec_steps(self.h)) * N
        T = _arr(L.orc_sim_rec_T(self.h), n, np.int32).reshape(-1, N)
        if self.arith == ARITH_INT32:
            w = _arr(L.orc_sim_rec_w(self.h), n, np.int64).reshape(-1, N)
        else:
            w = _arr(L.orc_sim_rec_w64(self.h), n, np.float64).reshape(-1, N)
        return T, w


def single_neuron(q, cfg: Optional[Config] = None, arith=ARITH_INT32):
    """Drive one synapse-less neuron with per-step input q; returns (U, I, R)."""
    cfg = cfg or Config()
    k = _consts_struct(cfg)
    n = len(q)
    r = np.zeros(n, np.int32)
    if arith == ARITH_INT32:
        qq = np.ascontiguousarray(q, dtype=np.int64)
        u = np.zeros(n, np.float32)
        i = np.zeros(n, np.float32)
        _check(lib().orc_single_neuron_f32(C.byref(k), qq.ctypes.data_as(C.POINTER(C.c_int64)), n,
                                           u.ctypes.data_as(C.POINTER(C.c_float)),
                                           i.ctypes.data_as(C.POINTER(C.c_float)),
                                           r.ctypes.data_as(C.POINTER(C.c_int32))))
    else:
        qq = np.ascontiguousarray(q, dtype=np.float64)
        u = np.zeros(n, np.float64)
        i = np.zeros(n, np.float64)
        _check(lib().orc_single_neuron_f64(C.byref(k), qq.ctypes.data_as(C.POINTER(C.c_double)), n,
                                           u.ctypes.data_as(C.POINTER(C.c_double)),
                                           i.ctypes.data_as(C.POINTER(C.c_double)),
                                           r.ctypes.data_as(C.POINTER(C.c_int32))))
    return u, i, r
