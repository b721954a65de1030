"""CPU-side checks of the simulator library (no GPU): the C ABI loads and
exports every function include/snn.h declares, argument validation fails
before any device work, and the host network sampler equals the oracle's."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def P():
    import paper_2405_02019_amd as P
    from paper_2405_02019_amd import build_lib
    if not os.path.exists(P.snn.LIB_PATH):
        build_lib.build()
    return P


def declared_functions():
    src = open(os.path.join(ROOT, "include", "snn.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(snn_\w+)\s*\(", src)))


def test_exports_every_declared_function(P):
    names = declared_functions()
    assert len(names) >= 12
    lib = P.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(P.snn.SIGNATURES)


def test_struct_layouts_match_header(P):
    """The binding's ctypes structures have the header's field count and a
    size consistent with the C layout (checked against offsets computed by a
    tiny C compile of the header)."""
    import subprocess
    import tempfile
    prog = r"""
#include <stdio.h>
#include <stddef.h>
#include "snn.h"
int main(void){printf("%zu %zu %zu %zu %zu\n", sizeof(snn_instance_cfg), sizeof(snn_config),
 sizeof(snn_state), sizeof(snn_info), sizeof(snn_host_network)); return 0;}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "s.c")
        open(c, "w").write(prog)
        exe = os.path.join(d, "s")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        sizes = [int(x) for x in subprocess.check_output([exe]).split()]
    S = P.snn
    assert sizes == [C.sizeof(S._Inst), C.sizeof(S._Cfg), C.sizeof(S._State), C.sizeof(S._Info),
                     C.sizeof(S._HostNet)]


def test_defaults(P):
    S = P.snn
    cfg = S._Cfg()
    P.lib().snn_config_default(C.byref(cfg))
    assert cfg.abi_version == S.ABI_VERSION and cfg.chunk_steps == 100 and cfg.use_graphs == 1
    inst = S._Inst()
    P.lib().snn_instance_default(C.byref(inst))
    assert inst.seed == 1 and inst.scale == 1.0 and inst.g == -4.0 and inst.bg_rate_hz == 8.0
    assert inst.psp_ext_mv == 0.15 and inst.bg_const_T == -1


def test_build_rejects_bad_configs_without_gpu(P):
    S = P.snn
    L = P.lib()
    h = C.c_void_p()
    cfg = S._Cfg()
    L.snn_config_default(C.byref(cfg))
    assert L.snn_build(C.byref(cfg), C.byref(h)) == -1          # no instances attached
    assert b"instances" in L.snn_last_error(None)
    inst = S._Inst()
    L.snn_instance_default(C.byref(inst))
    cfg.inst = C.pointer(inst)
    cfg.abi_version = 99
    assert L.snn_build(C.byref(cfg), C.byref(h)) == -1
    cfg.abi_version = S.ABI_VERSION
    cfg.syn_format = 7
    assert L.snn_build(C.byref(cfg), C.byref(h)) == -1
    assert not h
    assert L.snn_step_n(None, 1) == -1
    L.snn_destroy(None)


def test_per_instance_windows_are_checked_without_gpu(P):
    """Per-instance window lengths (load-balanced windows, Sec. 3.6's
    destination classes sized by their events): positive multiples of 4, for
    the LDS or banded engine, exclusive with window_neurons; all three are
    refused before any device call."""
    S = P.snn
    L = P.lib()
    h = C.c_void_p()
    insts = (S._Inst * 2)()
    for k in range(2):
        L.snn_instance_default(C.byref(insts[k]))
    cfg = S._Cfg()
    L.snn_config_default(C.byref(cfg))
    cfg.n_instances = 2
    cfg.inst = C.cast(insts, C.POINTER(S._Inst))
    each = (C.c_uint32 * 2)(256, 512)
    cfg.inst_window_neurons = C.cast(each, C.POINTER(C.c_uint32))
    cfg.engine = P.ENGINE_BAND
    cfg.window_neurons = 256
    assert L.snn_build(C.byref(cfg), C.byref(h)) == -1
    assert b"exclusive" in L.snn_last_error(None)
    cfg.window_neurons = 0
    cfg.engine = 0   # automatic choice
    assert L.snn_build(C.byref(cfg), C.byref(h)) == -1
    assert b"LDS or banded" in L.snn_last_error(None)
    cfg.engine = P.ENGINE_LDS
    each[1] = 258
    assert L.snn_build(C.byref(cfg), C.byref(h)) == -1
    assert b"instance 1: window length 258" in L.snn_last_error(None)
    assert not h


@pytest.mark.parametrize("fmt,wmode", [("plain", 0), ("compressed", 1)])
@pytest.mark.parametrize("scale,mode,seed", [(0.01, 0, 1), (0.05, 0, 9), (0.04, 1, 4)])
def test_sampler_equals_oracle(P, oracle, fmt, wmode, scale, mode, seed):
    """The library's sampler (C++, threaded two-pass counting sort) and the
    oracle's (C, sequential) build the same network: identical per-sender
    rows, delays, fixed-point weights and initial potentials."""
    a = P.sample_network(P.Instance(scale=scale, indegree_mode=mode, seed=seed), fmt)
    net = oracle.Net(oracle.Config(scale=scale, indegree_mode=mode, seed=seed, weight_mode=wmode))
    rp, post, d, w, wq = net.csr()
    assert a["n"] == net.N and a["nsyn"] == net.nsyn
    np.testing.assert_array_equal(a["pop_offset"], net.pop_offsets())
    np.testing.assert_array_equal(a["row_ptr"], rp)
    np.testing.assert_array_equal(a["u0"], net.u0())
    if fmt == "plain":
        np.testing.assert_array_equal(a["post"], post)
        np.testing.assert_array_equal(a["delay"], d)
        np.testing.assert_array_equal(a["w_q"], wq)
    else:   # compressed rows are grouped by 65,536-neuron target block
        pre = np.repeat(np.arange(net.N), np.diff(rp).astype(np.int64))
        k1 = np.lexsort((a["w_q"], a["delay"], a["post"], pre))
        k2 = np.lexsort((wq, d, post, pre))
        np.testing.assert_array_equal(a["post"][k1], post[k2])
        np.testing.assert_array_equal(a["delay"][k1], d[k2])
        np.testing.assert_array_equal(a["w_q"][k1], wq[k2])


@pytest.mark.parametrize("window", [256, 512])
@pytest.mark.parametrize("fmt,wmode", [("plain", 0), ("compressed", 1), ("dev8", 2)])
def test_windowed_layout_holds_the_oracle_network(P, oracle, window, fmt, wmode):
    """The LDS engine's layout (fixed-capacity segments per sender and target
    window, unused slots marked by delay 0) read back gives every row of the
    oracle's network, as a multiset, and nothing else."""
    scale, mode, seed = 0.04, 1, 4
    a = P.sample_network(P.Instance(scale=scale, indegree_mode=mode, seed=seed), fmt, window=window)
    net = oracle.Net(oracle.Config(scale=scale, indegree_mode=mode, seed=seed, weight_mode=wmode))
    rp, post, d, w, wq = net.csr()
    assert a["nsyn"] == net.nsyn
    np.testing.assert_array_equal(a["row_ptr"], rp)
    pre = np.repeat(np.arange(net.N), np.diff(rp).astype(np.int64))
    k1 = np.lexsort((a["w_q"], a["delay"], a["post"], pre))
    k2 = np.lexsort((wq, d, post, pre))
    np.testing.assert_array_equal(a["post"][k1], post[k2])
    np.testing.assert_array_equal(a["delay"][k1], d[k2])
    np.testing.assert_array_equal(a["w_q"][k1], wq[k2])
    # rows are ordered by target window
    win = a["post"].astype(np.int64) // window
    same_row = pre[1:] == pre[:-1]
    assert np.all(win[1:][same_row] >= win[:-1][same_row])
    with pytest.raises(P.SnnError, match="INVAL"):
        P.sample_network(P.Instance(scale=0.01), fmt, window=100)


@pytest.mark.parametrize("window,ring_rows", [(256, 64), (1000, 16), (2048, 8), (320, 32)])
@pytest.mark.parametrize("fmt,wmode", [("plain", 0), ("compressed", 1), ("dev8", 2)])
def test_banded_layout_holds_the_oracle_network(P, oracle, window, ring_rows, fmt, wmode):
    """The banded engine's layout (fixed-capacity segments per sender,
    target window and delay band: delay 1, then bands of H delays from 2 on,
    Sec. 3.4) read back gives every row of the oracle's network, as a
    multiset, and nothing else; within a row, synapses come by window, then
    by band, and every synapse sits in the band of its delay.  The deviation
    format's locators keep the delay relative to its band and the offset in
    its window, the pair's mean implicit (Sec. 5.3)."""
    scale, mode, seed = 0.04, 1, 4
    a = P.sample_network(P.Instance(scale=scale, indegree_mode=mode, seed=seed), fmt, window=window,
                         ring_rows=ring_rows)
    net = oracle.Net(oracle.Config(scale=scale, indegree_mode=mode, seed=seed, weight_mode=wmode))
    rp, post, d, w, wq = net.csr()
    assert a["nsyn"] == net.nsyn
    np.testing.assert_array_equal(a["row_ptr"], rp)
    pre = np.repeat(np.arange(net.N), np.diff(rp).astype(np.int64))
    k1 = np.lexsort((a["w_q"], a["delay"], a["post"], pre))
    k2 = np.lexsort((wq, d, post, pre))
    np.testing.assert_array_equal(a["post"][k1], post[k2])
    np.testing.assert_array_equal(a["delay"][k1], d[k2])
    np.testing.assert_array_equal(a["w_q"][k1], wq[k2])
    dl = a["delay"].astype(np.int64)
    band = np.where(dl <= 1, 0, 1 + (dl - 2) // ring_rows)
    key = (a["post"].astype(np.int64) // window) * 64 + band
    same_row = pre[1:] == pre[:-1]
    assert np.all(key[1:][same_row] >= key[:-1][same_row])
    assert band.max() <= (62 + ring_rows - 1) // ring_rows and band.max() >= 1


def test_dev8_format_is_for_the_lds_engines_only(P):
    """The deviation format (Sec. 5.3) is stored for the LDS and banded
    engines: the unwindowed layout and the other engines refuse it instead of
    quantising differently, and so do banded windows wider than its locator's
    offset field."""
    inst = P.Instance(scale=0.01)
    with pytest.raises(P.SnnError, match="INVAL"):
        P.sample_network(inst, "dev8")
    with pytest.raises(P.SnnError, match="RANGE"):
        P.sample_network(inst, "dev8", window=1024, ring_rows=64)   # 9 offset bits at 64 rows
    S = P.snn
    L = P.lib()
    h = C.c_void_p()
    cfg = S._Cfg()
    L.snn_config_default(C.byref(cfg))
    ci = S._Inst()
    L.snn_instance_default(C.byref(ci))
    cfg.inst = C.pointer(ci)
    cfg.syn_format = S.SYN_DEV8
    for engine in [S.ENGINE_PERSISTENT, S.ENGINE_STEPWISE]:
        cfg.engine = engine
        assert L.snn_build(C.byref(cfg), C.byref(h)) == -1   # checked before any device call
        assert b"LDS and banded engines only" in L.snn_last_error(None)
        assert not h


def test_banded_layout_rejects_bad_shapes(P):
    inst = P.Instance(scale=0.01)
    for window, rows in [(0, 16), (4098, 16), (255, 64), (256, 12), (256, 128)]:
        with pytest.raises(P.SnnError, match="INVAL"):
            P.sample_network(inst, "plain", window=window, ring_rows=rows)
    # compressed offsets take 16 - log2(H) bits: 1,024 neurons at H = 64
    with pytest.raises(P.SnnError, match="RANGE"):
        P.sample_network(inst, "compressed", window=2048, ring_rows=64)


def test_sampler_independent_of_thread_count(P):
    a = P.sample_network(P.Instance(scale=0.05, seed=2), "plain", host_threads=1)
    b = P.sample_network(P.Instance(scale=0.05, seed=2), "plain", host_threads=7)
    for k in ["row_ptr", "post", "delay", "w_q", "u0"]:
        np.testing.assert_array_equal(a[k], b[k])
    for fmt in ["plain", "compressed"]:
        a = P.sample_network(P.Instance(scale=0.05, seed=2), fmt, host_threads=1, window=700,
                             ring_rows=16)
        b = P.sample_network(P.Instance(scale=0.05, seed=2), fmt, host_threads=5, window=700,
                             ring_rows=16)
        for k in ["row_ptr", "post", "delay", "w_q", "u0"]:
            np.testing.assert_array_equal(a[k], b[k])


def test_sampler_error_paths(P):
    with pytest.raises(P.SnnError, match="OVERFLOW"):
        P.sample_network(P.Instance(scale=0.01, g=-50000.0))
    with pytest.raises(P.SnnError, match="RANGE"):
        P.sample_network(P.Instance(scale=0.01, g=-40.0), "compressed")
    with pytest.raises(P.SnnError, match="INVAL"):
        P.sample_network(P.Instance(scale=0.0))
    with pytest.raises(P.SnnError, match="INVAL"):
        P.sample_network(P.Instance(scale=0.01, conn=np.full(64, 1.5)))
    with pytest.raises(P.SnnError, match="INVAL"):
        P.sample_network(P.Instance(scale=0.01, bg_const_T=65))


def _windows(n, L):
    """Windows of an instance of n neurons at window length L (balanced
    windows of whole quads)."""
    nq = (n + 3) // 4
    nw = -(-nq // (L // 4))
    wq = -(-nq // nw)
    return -(-nq // wq)


def test_balanced_windows_reach_the_brute_force_optimum(P):
    """Windows sized by load (snn_balanced_windows; Sec. 3.6's destination
    classes, each block delivering about as many events): over every
    combination of window lengths (multiples of 4 up to the capacity) whose
    windows fit the blocks, the smallest possible maximum per-block load
    max_k load_k * L_k is what the bisection reaches, within its
    resolution."""
    import itertools
    rng = np.random.default_rng(3)
    for case in range(12):
        k = int(rng.integers(2, 4))
        n = [int(x) for x in rng.integers(20, 400, k)]
        load = [float(x) for x in rng.uniform(0.2, 3.0, k)]
        wn = int(rng.choice([32, 64, 96]))
        fewest = sum(_windows(nk, wn) for nk in n)
        blocks = fewest + int(rng.integers(0, 12))
        L = P.balanced_windows(n, load, wn, blocks)
        assert all(4 <= x <= wn and x % 4 == 0 for x in L)
        assert sum(_windows(nk, x) for nk, x in zip(n, L)) <= blocks
        best = min(max(w * x for w, x in zip(load, combo))
                   for combo in itertools.product(range(4, wn + 1, 4), repeat=k)
                   if sum(_windows(nk, x) for nk, x in zip(n, combo)) <= blocks)
        got = max(w * x for w, x in zip(load, L))
        assert got <= best * (1 + 1e-9), (case, n, load, wn, blocks, L, got, best)


def test_balanced_windows_special_cases(P):
    """Equal instances get equal windows; an instance with twice the load
    gets about half the window; a silent one the full capacity; the
    capacity itself when the blocks allow nothing shorter; errors for
    windows that cannot fit and for bad arguments."""
    assert P.balanced_windows([1000, 1000], [1.0, 1.0], 512, 8) == [252, 252]
    a, b = P.balanced_windows([1000, 1000], [1.0, 2.0], 512, 12)
    assert abs(a / b - 2.0) < 0.1
    assert P.balanced_windows([1000, 1000], [0.0, 1.0], 512, 64)[0] == 512
    assert P.balanced_windows([1000], [1.0], 512, 2) == [500]
    assert P.balanced_windows([1024], [1.0], 512, 2) == [512]
    with pytest.raises(P.SnnError, match="RANGE"):
        P.balanced_windows([1024], [1.0], 512, 1)
    with pytest.raises(P.SnnError, match="INVAL"):
        P.balanced_windows([1000], [-1.0], 512, 8)
    with pytest.raises(P.SnnError, match="INVAL"):
        P.balanced_windows([1000], [1.0], 510, 8)
