"""The request loop (``serve.run_stream``) and the server's argument checks
without a GPU: a fake server that finishes each shot a fixed time after
admission, with a slot limit, stands in for the device."""
import ctypes as C
import time

import numpy as np
import pytest

import synth
from paper_2205_07976_amd import serve, xrt


class FakeInfo:
    def __init__(self, state, t_submit, t_admit, t_done):
        self.state, self.t_submit, self.t_admit, self.t_done = state, t_submit, t_admit, t_done


class FakeServer:
    """Admits in arrival order up to `slots`; a shot is done `service` s after
    admission."""

    def __init__(self, slots=2, service=0.004):
        self.slots, self.service = slots, service
        self.t0 = time.perf_counter()
        self.shots = {}
        self.queue = []
        self.next = 1
        self.admit_order = []

    def now(self):
        return time.perf_counter() - self.t0

    def submit(self, shot):
        t = self.next
        self.next += 1
        self.shots[t] = {"submit": self.now(), "admit": -1.0, "done": -1.0}
        self.queue.append(t)
        return t

    def progress(self):
        """As xrt_server_progress: returns the number of shots seen finishing
        in this call."""
        now = self.now()
        n_done = 0
        for t, s in self.shots.items():
            if s["admit"] >= 0 and s["done"] < 0 and now - s["admit"] >= self.service:
                s["done"] = now
                n_done += 1
        running = sum(1 for s in self.shots.values() if s["admit"] >= 0 and s["done"] < 0)
        while self.queue and running < self.slots:
            t = self.queue.pop(0)
            self.shots[t]["admit"] = now
            self.admit_order.append(t)
            running += 1
        return n_done

    def info(self, t):
        s = self.shots[t]
        return FakeInfo(2 if s["done"] >= 0 else (1 if s["admit"] >= 0 else 0), s["submit"], s["admit"], s["done"])

    def image(self, t):
        return t

    def release(self, t):
        assert self.shots[t]["done"] >= 0
        del self.shots[t]


def test_run_stream_with_fake_server():
    shots = [synth.tiny_shot()] * 20
    srv = FakeServer(slots=2, service=0.004)
    arr = serve.poisson_arrivals(np.random.default_rng(0), len(shots), rate=200.0)
    res = serve.run_stream(srv, shots, arr, keep=[3])
    assert srv.admit_order == sorted(srv.admit_order)  # arrival order
    assert np.all(res["latency"] >= 0.004 - 1e-6)
    assert res["images"][3] == res["tickets"][3]
    st = serve.summarize(res, shots, 200.0)
    assert st["shots"] == 20 and st["p99_ms"] >= st["p50_ms"] >= 4.0
    assert not srv.shots  # everything released


class FakeWriteOutServer(FakeServer):
    """The fake server with write-out: images are host arrays."""
    writes_out = True

    def host_image(self, t):
        assert self.shots[t]["done"] >= 0
        return np.full((2, 3), float(t))


@pytest.mark.parametrize("writers", [0, 3])
def test_run_stream_sinks_every_image_then_releases(writers):
    """Every finished shot's host image reaches the sink exactly once, before
    its release, in the loop or on writer threads."""
    import threading
    shots = [synth.tiny_shot()] * 15
    srv = FakeWriteOutServer(slots=3, service=0.002)
    seen, lock = {}, threading.Lock()

    def sink(i, img):
        time.sleep(0.003)  # a slow writer
        with lock:
            assert i not in seen
            seen[i] = img

    res = serve.run_stream(srv, shots, np.zeros(len(shots)), sink=sink, writers=writers)
    assert sorted(seen) == list(range(15))
    for i, img in seen.items():
        assert np.all(img == res["tickets"][i])
    assert not srv.shots


def test_poisson_arrivals_rate():
    a = serve.poisson_arrivals(np.random.default_rng(2), 20000, rate=50.0)
    assert np.all(np.diff(a) > 0)
    assert abs(len(a) / a[-1] - 50.0) < 1.5


@pytest.mark.parametrize("field,value,code", [
    ("hbm_budget", 1000, xrt.XRT_ERANGE),
    ("max_resident", 0, xrt.XRT_ERANGE),
    ("precision", 5, xrt.XRT_EINVAL),
    ("shape", 3, xrt.XRT_EINVAL),
    ("idle_exit_us", 0.0, xrt.XRT_ERANGE),
    ("policy", 2, xrt.XRT_EINVAL),
])
def test_server_desc_validation(field, value, code):
    d = xrt.ServerDesc(C.sizeof(xrt.ServerDesc), 1 << 30, 16, xrt.XRT_MIXED, 0, xrt.XRT_F32, 0, 1000.0)
    setattr(d, field, value)
    h = C.c_void_p()
    assert xrt.load().xrt_server_create(C.byref(d), C.c_void_p(1), C.byref(h)) == code
    assert not h.value
