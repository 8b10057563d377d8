"""Served shots with write-out (a host budget): every image arrives in the
server's pinned host memory bit-identical to the standalone kernel's; a shot's
device memory and resident slot are freed when its copy completes, without a
release by the client; host memory applies back-pressure; misuse is refused."""
import sys
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2205_07976_amd import serve, xrt  # noqa: E402
from tests.test_gpu_serve import small_served_shots  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def progress_until(server, pred, timeout=60.0):
    t0 = time.time()
    while not pred():
        server.progress()
        if time.time() - t0 > timeout:
            raise TimeoutError("condition not reached")


def states(server, tickets):
    return [server.info(t).state for t in tickets]


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_written_out_equal_standalone(precision):
    base, shots = small_served_shots(10, seed=51)
    fh = xrt.Fhkl.from_shot(base)
    srv = xrt.Server(fh, hbm_budget=256 << 20, max_resident=8, precision=precision, host_budget=64 << 20)
    res = serve.run_stream(srv, shots, np.zeros(len(shots)), keep=range(len(shots)))
    for i, s in enumerate(shots):
        ref = xrt.simulate(s, fh, precision=precision).cpu().numpy()
        assert np.array_equal(res["images"][i], ref), i
    t = srv.submit(shots[0])
    progress_until(srv, lambda: srv.info(t).state == xrt.XRT_SHOT_DONE)
    with pytest.raises(xrt.XrtError) as e:
        srv.image(t)  # images live on the host
    assert e.value.code == xrt.XRT_EINVAL
    with pytest.raises(xrt.XrtError) as e:
        srv.cancel(t)  # done
    assert e.value.code == xrt.XRT_EBUSY
    srv.release(t)
    srv.close()


def test_slots_freed_when_the_copy_completes():
    """One resident slot and a client that releases nothing: with write-out
    every shot still runs (each copy frees the slot); without it the first
    shot keeps the slot and the others stay queued."""
    base, shots = small_served_shots(5, seed=52)
    fh = xrt.Fhkl.from_shot(base)
    srv = xrt.Server(fh, hbm_budget=256 << 20, max_resident=1, precision="mixed", host_budget=64 << 20)
    tickets = [srv.submit(s) for s in shots]
    progress_until(srv, lambda: all(st == xrt.XRT_SHOT_DONE for st in states(srv, tickets)))
    for t, s in zip(tickets, shots):
        assert np.array_equal(srv.host_image(t), xrt.simulate(s, fh, precision="mixed").cpu().numpy())
        srv.release(t)
    srv.close()

    srv = xrt.Server(fh, hbm_budget=256 << 20, max_resident=1, precision="mixed")
    tickets = [srv.submit(s) for s in shots]
    progress_until(srv, lambda: srv.info(tickets[0]).state == xrt.XRT_SHOT_DONE)
    for _ in range(200):
        srv.progress()
    st = states(srv, tickets)
    say("in place, nothing released:", st)
    assert st[0] == xrt.XRT_SHOT_DONE and all(x == xrt.XRT_SHOT_QUEUED for x in st[1:])
    srv.release(tickets[0])
    srv.close()


def test_host_memory_back_pressure():
    """A 1 MiB host budget holds at most four 230 x 250 binary32 images: the
    rest wait on the device, finished but not copied, until releases make
    room; every image still arrives intact."""
    base, shots = small_served_shots(7, seed=53)
    shots = [s.replace(roi=(s.roi[0], s.roi[0] + 230, s.roi[2], s.roi[2] + 250)) if s.roi[0] + 230 <= 2463
             and s.roi[2] + 250 <= 2527 else s.replace(roi=(0, 230, 0, 250)) for s in shots]
    fh = xrt.Fhkl.from_shot(base)
    srv = xrt.Server(fh, hbm_budget=256 << 20, max_resident=16, precision="mixed", host_budget=1 << 20)
    tickets = [srv.submit(s) for s in shots]
    t0 = time.time()
    while time.time() - t0 < 10.0:
        srv.progress()
        if sum(x == xrt.XRT_SHOT_DONE for x in states(srv, tickets)) == 4:
            break
    for _ in range(300):
        srv.progress()
    st = states(srv, tickets)
    say("host budget full:", st)
    assert sum(x == xrt.XRT_SHOT_DONE for x in st) == 4
    assert all(x == xrt.XRT_SHOT_RUNNING for x in st if x != xrt.XRT_SHOT_DONE)
    done = set()
    while len(done) < len(tickets):
        srv.progress()
        for t, s in zip(tickets, shots):
            if t not in done and srv.info(t).state == xrt.XRT_SHOT_DONE:
                assert np.array_equal(srv.host_image(t), xrt.simulate(s, fh, precision="mixed").cpu().numpy())
                srv.release(t)
                done.add(t)
    srv.close()


def test_image_larger_than_host_budget_refused():
    base, shots = small_served_shots(1, seed=54)
    fh = xrt.Fhkl.from_shot(base)
    srv = xrt.Server(fh, hbm_budget=256 << 20, max_resident=4, precision="mixed", host_budget=1 << 20)
    big = shots[0].replace(roi=(0, 700, 0, 700))  # 1.96 MB of binary32
    with pytest.raises(xrt.XrtError) as e:
        srv.submit(big)
    assert e.value.code == xrt.XRT_ERANGE
    srv.close()
