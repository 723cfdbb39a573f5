"""Distinct contexts used from different threads at once: each thread
creates, tunes, steps and reads back its own context (the library's only
shared state is the process-wide cache of tuned tile shapes).  The results
must equal the same work done serially, bit for bit.  ctypes releases the
interpreter lock during each library call, so the calls do overlap."""
import threading

import numpy as np
import pytest

from parity_util import small_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_1402_2920_amd import lb2p
    lb2p.lib()
    return lb2p


def _work(L, lattice, shape, seed):
    rho, u, m = small_case(lattice, shape, seed=seed)
    P = L.Params(lattice=lattice, nx=shape[0], ny=shape[1], nz=shape[2] if len(shape) == 3 else 1,
                 storage=L.STORE_F32, gamma=m["gamma"], kappa=m["kappa"], rho1=m["rho1"], rho2=m["rho2"],
                 A=m["A"], cs2_rho1=m["cs2_1"], rho0=m["rho0"], tol=1e-6, max_iter=500)
    with L.Context(P) as ctx:
        ctx.init(rho, u)
        ctx.autotune(1)
        ctx.step(5)
        r, uu = ctx.moments()
    return r, uu


CASES = [(21, (40, 24), 31), (59, (20, 12, 10), 32), (21, (72, 20), 33), (59, (24, 16, 12), 34)]


def test_contexts_on_threads_match_serial(L):
    serial = [_work(L, *c) for c in CASES]
    out = [None] * len(CASES)
    errs = []

    def run(k):
        try:
            out[k] = _work(L, *CASES[k])
        except Exception as ex:   # reported below, with the case
            errs.append((CASES[k], repr(ex)))

    th = [threading.Thread(target=run, args=(k,)) for k in range(len(CASES))]
    for t in th:
        t.start()
    for t in th:
        t.join(timeout=300)
    assert not errs, errs
    assert all(not t.is_alive() for t in th)
    for k, c in enumerate(CASES):
        print("case", c, "threaded == serial", flush=True)
        np.testing.assert_array_equal(out[k][0], serial[k][0])
        np.testing.assert_array_equal(out[k][1], serial[k][1])
