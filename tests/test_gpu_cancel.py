"""Cancellation (kc_opts.cancel -> KC_ECANCELED) and its absence.

A flag that is already set stops every traversal path at once; a cleared flag
changes nothing; a flag set by a host thread while a long count runs stops it
early.  Every kernel exits normally in all cases: the flag only makes them stop
taking work.
"""
import ctypes
import threading
import time

import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

HIP_HOST_MALLOC_MAPPED = 0x2
HIP_HOST_MALLOC_COHERENT = 0x40000000


class HostFlag:
    """One int32 of pinned, device-mapped, coherent host memory."""

    def __init__(self):
        import torch  # noqa: F401  (loads the HIP runtime this process uses)
        self.hip = ctypes.CDLL("libamdhip64.so.7")
        self.hip.hipHostMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t, ctypes.c_uint]
        self.hip.hipHostFree.argtypes = [ctypes.c_void_p]
        p = ctypes.c_void_p()
        assert self.hip.hipHostMalloc(ctypes.byref(p), 64, HIP_HOST_MALLOC_MAPPED | HIP_HOST_MALLOC_COHERENT) == 0
        self.addr = p.value
        self.set(0)

    def set(self, v):
        ctypes.c_int32.from_address(self.addr).value = v

    def free(self):
        self.hip.hipHostFree(ctypes.c_void_p(self.addr))


@pytest.fixture(scope="module")
def flag():
    f = HostFlag()
    yield f
    f.free()


@pytest.fixture(scope="module")
def graphs(kc):
    out = {}
    for name, g in (("chung_lu", synth.chung_lu(4000, 2.1, 24.0, 600.0, 5)),
                    ("heavy_core", synth.dense_core(5000, 8.0, 2.1, 3, 150, 260, 0.45, 7))):
        out[name] = (g, kc.orient(kc.to_device(g), kc.ORDER_DEGENERACY))
    return out


CASES = [  # (graph, k, pivot, scheme, width): lane walk, deep lane walk, group walk, pivot
    ("chung_lu", 5, False, 1, 0),
    ("heavy_core", 8, False, 2, 0),
    ("heavy_core", 6, False, 1, 8),
    ("chung_lu", 5, True, 1, 0),
    ("heavy_core", 7, True, 2, 0),
]


@pytest.mark.parametrize("case", CASES)
def test_set_flag_cancels_and_cleared_flag_counts(kc, graphs, flag, case):
    name, k, pivot, scheme, width = case
    g, d = graphs[name]
    print("cancel: %s k=%d pivot=%d scheme=%d width=%d" % case, flush=True)
    flag.set(1)
    st, _ = kc.count_status(d, k, pivot, scheme, width, cancel=flag.addr)
    assert st == kc.ECANCELED
    flag.set(0)
    st, got = kc.count_status(d, k, pivot, scheme, width, cancel=flag.addr)
    assert st == kc.OK
    assert got == oracle.count(oracle.orient(g, oracle.DEGENERACY), k, False, oracle.EC)


@pytest.mark.parametrize("pivot", [True, False])
def test_count_all_cancel(kc, graphs, flag, pivot):
    g, d = graphs["heavy_core"]
    flag.set(1)
    st, _, _ = kc.count_all_status(d, pivot=pivot, cancel=flag.addr)
    assert st == kc.ECANCELED
    flag.set(0)
    st, got, om = kc.count_all_status(d, pivot=pivot, cancel=flag.addr)
    want, wom = oracle.count_all(oracle.orient(g, oracle.DEGENERACY), True, oracle.VC)
    assert st == kc.OK and om == wom
    assert got[:om + 1] == want[:om + 1]


def test_device_memory_flag(kc, graphs):
    import torch
    g, d = graphs["chung_lu"]
    f = torch.ones(1, dtype=torch.int32, device="cuda")
    st, _ = kc.count_status(d, 5, cancel=f.data_ptr())
    assert st == kc.ECANCELED
    f.zero_()
    st, got = kc.count_status(d, 5, cancel=f.data_ptr())
    assert st == kc.OK and got == kc.count(d, 5)


@pytest.mark.parametrize("pivot", [False, True])
def test_cancel_while_running(kc, flag, pivot):
    # the dense-core workload: non-pivot k = 13 with edge roots and pivot
    # count-all each run for seconds; a host thread raises the flag after 0.2 s
    g = synth.config_densecore()
    d = kc.orient(kc.to_device(g), kc.ORDER_DEGENERACY)
    flag.set(0)
    timer = threading.Timer(0.2, flag.set, args=(1,))
    t0 = time.perf_counter()
    timer.start()
    if pivot:
        st, _, _ = kc.count_all_status(d, pivot=True, scheme=kc.SCHEME_VC, cancel=flag.addr)
    else:
        st, _ = kc.count_status(d, 13, False, kc.SCHEME_EC, cancel=flag.addr)
    dt = time.perf_counter() - t0
    timer.join()
    flag.set(0)
    print("cancel while running: pivot=%d status=%d after %.3f s" % (pivot, st, dt), flush=True)
    assert st == kc.ECANCELED
    assert dt < 1.0
