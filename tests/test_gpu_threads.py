"""Stateless entry points called from several host threads at once, each on
its own stream: every thread's results equal the single-threaded ones, and
the error message a thread reads is the one its own failed call left."""
import threading

import pytest
import torch

from gpu_util import dev, need_gpu
from paper_1804_10120_amd import TLError, tl_dtg_chain, tl_dtg_chain_bwd
from paper_1804_10120_amd.synth import make_fields

pytestmark = pytest.mark.gpu

KEYS = ("g", "dg", "beta", "dbeta", "K", "alpha")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def test_concurrent_calls_on_separate_streams():
    nthreads, reps = 6, 20
    cases = []
    for t in range(nthreads):
        n = 1000 + 4099 * t
        f = make_fields(n, seed=500 + t)
        d = {k: dev(f[k]) for k in KEYS + ("W",)}
        ref_f = tl_dtg_chain(*[d[k] for k in KEYS])
        ref_b = tl_dtg_chain_bwd(d["g"], d["dg"], d["beta"], d["K"], d["alpha"], d["W"])
        cases.append((d, ref_f, ref_b))
    torch.cuda.synchronize()
    errors, barrier = [], threading.Barrier(nthreads)

    def work(t):
        try:
            d, ref_f, ref_b = cases[t]
            stream = torch.cuda.Stream()
            barrier.wait()
            with torch.cuda.stream(stream):
                for r in range(reps):
                    out = tl_dtg_chain(*[d[k] for k in KEYS])
                    grads = tl_dtg_chain_bwd(d["g"], d["dg"], d["beta"], d["K"], d["alpha"],
                                             d["W"])
                    # a failing call between good ones, with a different error in
                    # odd and even threads: each must read its own message
                    with pytest.raises(TLError) as e:
                        if t % 2:
                            tl_dtg_chain(*[d[k] for k in KEYS], dtg=d["K"])
                        else:
                            tl_dtg_chain(*[d[k] for k in KEYS], tune=dict(block=96))
                    msg = str(e.value)
                    if t % 2:
                        assert "overlaps" in msg and "dtg" in msg and "K" in msg, msg
                    else:
                        assert "tune.block=96" in msg, msg
                stream.synchronize()
            assert torch.equal(out, ref_f), f"thread {t}: d_t g"
            for a, b in zip(grads, ref_b):
                assert torch.equal(a, b), f"thread {t}: gradient"
        except BaseException as e:       # reported by the main thread
            errors.append((t, repr(e)))

    threads = [threading.Thread(target=work, args=(t,)) for t in range(nthreads)]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=120)
    assert not any(th.is_alive() for th in threads)
    assert errors == []
