"""Served shots (continuous batching in a persistent kernel) through the C ABI:
every image equals the standalone kernel's bit for bit, alone and in the mix;
admission follows the HBM budget in arrival order; oversized shots are
refused; the server relaunches its kernel after an idle exit."""
import sys
import time

import numpy as np
import pytest

import synth
from oracle import oracle as o
from tests.metrics import DBL_MIN, compare

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2205_07976_amd import serve, xrt  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def small_served_shots(n, seed=44, max_side=160):
    """Served-stream shots with small ROIs (the full-size detector and table,
    random orientation, sources, domains and N), so tests stay short."""
    base = synth.full_shot()
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        s = synth.served_shot(rng, base.F, base.hkl_min)
        wf, ws = int(rng.integers(8, max_side)), int(rng.integers(8, max_side))
        f0, s0 = int(rng.integers(0, 2463 - wf)), int(rng.integers(0, 2527 - ws))
        n_src = int(rng.integers(1, 9))
        n_mos = int(rng.integers(1, 17))
        s = s.replace(roi=(f0, f0 + wf, s0, s0 + ws), src_dir=s.src_dir[:n_src].copy(),
                      src_lambda=s.src_lambda[:n_src].copy(),
                      src_weight=s.src_weight[:n_src] / s.src_weight[:n_src].sum(),
                      umats=s.umats[:n_mos].copy())
        out.append(s)
    return base, out


def drain(server, tickets, timeout=60.0):
    t0 = time.time()
    while True:
        server.progress()
        states = [server.info(t).state for t in tickets]
        if all(st == xrt.XRT_SHOT_DONE for st in states):
            return
        if time.time() - t0 > timeout:
            raise TimeoutError(f"states {states}")


@pytest.mark.parametrize("precision,policy", [("mixed", "shortest_remaining"), ("fp64", "shortest_remaining"),
                                              ("mixed", "fair_share"), ("fp64", "fair_share")])
def test_served_equal_standalone_in_mix_and_alone(precision, policy):
    """Ten shots at once (they share the persistent kernel, in the order of
    either publication policy), then four alone: every image equals the
    standalone call's bit for bit."""
    base, shots = small_served_shots(10)
    fh = xrt.Fhkl.from_shot(base)
    ref = [xrt.simulate(s, fh, precision=precision).cpu().numpy() for s in shots]
    srv = xrt.Server(fh, hbm_budget=256 << 20, precision=precision, policy=policy)
    tickets = [srv.submit(s) for s in shots]  # all at once: they share the kernel
    drain(srv, tickets)
    for i, t in enumerate(tickets):
        img = srv.image(t).cpu().numpy()
        assert np.array_equal(img, ref[i]), f"shot {i} differs in the mix"
        srv.release(t)
    for i, s in enumerate(shots[:4]):  # alone, one after the other
        t = srv.submit(s)
        drain(srv, [t])
        assert np.array_equal(srv.image(t).cpu().numpy(), ref[i]), f"shot {i} differs alone"
        srv.release(t)
    srv.close()


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_served_short_rotation_lists(precision):
    """The served kernel reads the next spindle x domain matrix into the
    registers of the current one as soon as the current term's h is formed
    (the last term rereads its own): lists of 1 to 6 matrices, from domains
    alone and from spindle steps x domains, give the standalone images bit
    for bit."""
    base, shots = small_served_shots(8, seed=45, max_side=40)
    cases = [(1, 1), (2, 1), (3, 1), (4, 1), (1, 2), (3, 2), (2, 2), (1, 3)]  # (domains, spindle steps)
    shots = [s.replace(umats=s.umats[:1].repeat(m, axis=0) if len(s.umats) < m else s.umats[:m].copy(),
                       n_phi=k, phi0=0.01, dphi=0.02) for s, (m, k) in zip(shots, cases)]
    assert sorted(len(s.umats) * s.n_phi for s in shots) == [1, 2, 2, 3, 3, 4, 4, 6]
    fh = xrt.Fhkl.from_shot(base)
    ref = [xrt.simulate(s, fh, precision=precision).cpu().numpy() for s in shots]
    srv = xrt.Server(fh, hbm_budget=64 << 20, precision=precision)
    tickets = [srv.submit(s) for s in shots]
    drain(srv, tickets)
    for i, t in enumerate(tickets):
        assert np.array_equal(srv.image(t).cpu().numpy(), ref[i]), f"rotation list {cases[i]} differs"
        srv.release(t)
    srv.close()


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_served_gaussian_shape(precision):
    """A server of the Gaussian shape (real N, the refinement crystal's
    lattice form): every image equals the standalone Gaussian kernel's bit
    for bit in the mix, and matches the oracle on one small shot."""
    base, shots = small_served_shots(6, seed=61)
    rng = np.random.default_rng(62)
    shots = [s.replace(shape=synth.SHAPE_GAUSS, N=rng.uniform(5.0, 40.0, 3)) for s in shots]
    fh = xrt.Fhkl.from_shot(base)
    ref = [xrt.simulate(s, fh, precision=precision).cpu().numpy() for s in shots]
    srv = xrt.Server(fh, hbm_budget=256 << 20, precision=precision, shape=xrt.XRT_SHAPE_GAUSS)
    tickets = [srv.submit(s) for s in shots]
    drain(srv, tickets)
    for i, t in enumerate(tickets):
        assert np.array_equal(srv.image(t).cpu().numpy(), ref[i]), f"shot {i} differs in the mix"
        srv.release(t)
    srv.close()
    small = shots[0].replace(roi=(shots[0].roi[0], shots[0].roi[0] + 12, shots[0].roi[2], shots[0].roi[2] + 10))
    img = xrt.simulate(small, fh, precision=precision, out_dtype=torch.float64).cpu().numpy()
    ref = o.simulate(small)
    tol = 1e-12 if precision == "fp64" else 1e-5
    r = compare(img, ref, tiny=DBL_MIN)
    say("gauss served-shot oracle", precision, r)
    assert r["zeros_ok"] and r["max_rel"] <= tol and r["sub_abs"] <= tol


def test_served_binary64_images_of_mixed_sums():
    """A mixed-precision server with binary64 images stores the same sums
    the standalone kernel stores into a binary64 image."""
    base, shots = small_served_shots(4, seed=63)
    fh = xrt.Fhkl.from_shot(base)
    srv = xrt.Server(fh, hbm_budget=256 << 20, precision="mixed", out_dtype="f64")
    tickets = [srv.submit(s) for s in shots]
    drain(srv, tickets)
    for s, t in zip(shots, tickets):
        img = srv.image(t)
        assert img.dtype == torch.float64
        ref = xrt.simulate(s, fh, precision="mixed", out_dtype=torch.float64)
        assert torch.equal(img, ref)
        srv.release(t)
    srv.close()


def test_served_matches_oracle():
    base, shots = small_served_shots(3, seed=7, max_side=40)
    fh = xrt.Fhkl.from_shot(base)
    srv = xrt.Server(fh, hbm_budget=64 << 20, precision="mixed")
    tickets = [srv.submit(s) for s in shots]
    drain(srv, tickets)
    for s, t in zip(shots, tickets):
        r = compare(srv.image(t).cpu().numpy(), o.simulate(s))
        say(s.roi, r)
        assert r["zeros_ok"] and r["max_rel"] <= 1e-5
    srv.close()


def test_admission_by_budget_in_arrival_order():
    """A 3 MiB budget holds at most two of these shots (about 1.2 MiB each):
    the others wait, admissions follow arrival order, and all finish."""
    base, shots = small_served_shots(7, seed=3, max_side=20)
    shots = [s.replace(roi=(100 + 5 * i, 100 + 5 * i + 560, 200, 200 + 560)) for i, s in enumerate(shots)]
    fh = xrt.Fhkl.from_shot(base)
    srv = xrt.Server(fh, hbm_budget=3 << 20, precision="mixed")
    tickets = [srv.submit(s) for s in shots]
    peak = 0
    t0 = time.time()
    while True:
        srv.progress()
        infos = [srv.info(t) for t in tickets]
        resident = sum(1 for i in infos if i.state == xrt.XRT_SHOT_RUNNING)
        peak = max(peak, resident)
        for t, i in zip(tickets, infos):
            if i.state == xrt.XRT_SHOT_DONE and i.t_done >= 0:
                pass
        done = [t for t, i in zip(tickets, infos) if i.state == xrt.XRT_SHOT_DONE]
        for t in done:
            srv.release(t)
            tickets.remove(t)
        if not tickets:
            break
        assert time.time() - t0 < 120
    say("peak resident", peak)
    assert 1 <= peak <= 2
    srv.close()


def test_refusals():
    base, shots = small_served_shots(1)
    fh = xrt.Fhkl.from_shot(base)
    srv = xrt.Server(fh, hbm_budget=1 << 20, precision="mixed")
    with pytest.raises(xrt.XrtError) as e:  # 2463 x 2527 x 4 B image > 1 MiB
        srv.submit(shots[0].replace(roi=(0, 2463, 0, 2527)))
    assert e.value.code == xrt.XRT_ERANGE
    many = shots[0].replace(src_dir=np.repeat(shots[0].src_dir[:1], 200, 0),
                            src_lambda=np.full(200, 1.3), src_weight=np.full(200, 1 / 200))
    with pytest.raises(xrt.XrtError) as e:
        srv.submit(many)
    assert e.value.code == xrt.XRT_ERANGE
    with pytest.raises(xrt.XrtError) as e:
        srv.submit(shots[0].replace(shape=synth.SHAPE_GAUSS))
    assert e.value.code == xrt.XRT_EINVAL
    srv.close()


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_full_shot_region_default_segments(precision):
    """A 1024 x 512 region of the full-size shot (2048 tiles, whole sums;
    100 sources, 50 domains, 60 000 terms per pixel) on a server with the
    default segment size, where every tile's sum runs as several consecutive
    segments: the image equals the standalone call's bit for bit."""
    shot = synth.full_shot().replace(roi=(700, 1724, 1000, 1512))
    segs = expected_segments(shot, 1 << 21)
    say("full-shot region: segments per tile", segs)
    assert segs > 1 and expected_split(shot) == 1
    fh = xrt.Fhkl.from_shot(shot)
    ref = xrt.simulate(shot, fh, precision=precision).cpu().numpy()
    srv = xrt.Server(fh, hbm_budget=256 << 20, precision=precision)
    t = srv.submit(shot)
    drain(srv, [t])
    assert np.array_equal(srv.image(t).cpu().numpy(), ref)
    srv.release(t)
    srv.close()


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_served_at_the_limits(precision):
    """A shot at the served limits (128 sources, 2 spindle steps x 128
    domains = 256 matrices: the largest tables a workgroup stages in LDS),
    on a ragged 23 x 19 region, beside a small one: bit for bit the
    standalone images; one source or one matrix more is refused."""
    base, shots = small_served_shots(2, seed=101)
    rng = np.random.default_rng(102)
    big = synth.served_shot(rng, base.F, base.hkl_min)
    lam, w = synth.shots.gaussian_spectrum(rng, 128, 1.30, 0.003)
    f0, s0 = 1200, 1250
    big = big.replace(roi=(f0, f0 + 23, s0, s0 + 19), src_dir=synth.shots.on_axis_sources(128), src_lambda=lam,
                      src_weight=w, umats=synth.shots.mosaic_umats(rng, 128, 0.05), n_phi=2, phi0=0.0, dphi=0.01)
    assert big.n_src == 128 and big.n_phi * big.n_mos == 256
    todo = [big, shots[0]]
    fh = xrt.Fhkl.from_shot(base)
    ref = [xrt.simulate(x, fh, precision=precision).cpu().numpy() for x in todo]
    srv = xrt.Server(fh, hbm_budget=64 << 20, precision=precision)
    tickets = [srv.submit(x) for x in todo]
    drain(srv, tickets)
    for i, t in enumerate(tickets):
        assert np.array_equal(srv.image(t).cpu().numpy(), ref[i]), f"shot {i} differs"
        srv.release(t)
    more_src = big.replace(src_dir=synth.shots.on_axis_sources(129), src_lambda=np.full(129, 1.3),
                           src_weight=np.full(129, 1.0 / 129))
    more_rot = big.replace(umats=np.concatenate([big.umats, big.umats[:1]]))
    for x in (more_src, more_rot):
        with pytest.raises(xrt.XrtError) as e:
            srv.submit(x)
        assert e.value.code == xrt.XRT_ERANGE
    srv.close()


def test_relaunch_after_idle_exit():
    base, shots = small_served_shots(4, seed=9, max_side=48)
    fh = xrt.Fhkl.from_shot(base)
    ref = [xrt.simulate(s, fh, precision="mixed").cpu().numpy() for s in shots]
    srv = xrt.Server(fh, hbm_budget=64 << 20, precision="mixed", idle_exit_us=500.0)
    for i, s in enumerate(shots):
        t = srv.submit(s)
        drain(srv, [t])
        assert np.array_equal(srv.image(t).cpu().numpy(), ref[i])
        srv.release(t)
        time.sleep(0.02)  # longer than the idle exit: the next shot needs a new kernel
    srv.close()


def test_kept_copy_survives_release_and_reuse():
    """A copy of a finished image taken by Server.image (default copy=True)
    is complete when the call returns: the shot is released at once, the next
    shot is admitted into the freed region (first fit: the same offset) and
    the persistent kernel writes it, and the kept copy still equals the
    standalone image bit for bit."""
    base, shots = small_served_shots(2, seed=17, max_side=96)
    a = shots[0]
    b = shots[1].replace(roi=(a.roi[0], a.roi[1], a.roi[2], a.roi[3]))  # same footprint
    fh = xrt.Fhkl.from_shot(base)
    ref = xrt.simulate(a, fh, precision="mixed").cpu().numpy()
    srv = xrt.Server(fh, hbm_budget=8 << 20, max_resident=1, precision="mixed")
    ta = srv.submit(a)
    drain(srv, [ta])
    pa = srv.image(ta, copy=False).data_ptr()
    kept = srv.image(ta)
    srv.release(ta)
    tb = srv.submit(b)
    drain(srv, [tb])
    assert srv.image(tb, copy=False).data_ptr() == pa  # b was written over a's region
    assert np.array_equal(kept.cpu().numpy(), ref)
    srv.release(tb)
    srv.close()


def test_run_stream_poisson():
    base, shots = small_served_shots(24, seed=12, max_side=96)
    fh = xrt.Fhkl.from_shot(base)
    srv = xrt.Server(fh, hbm_budget=256 << 20, precision="mixed")
    arr = serve.poisson_arrivals(np.random.default_rng(1), len(shots), rate=400.0)
    res = serve.run_stream(srv, shots, arr, keep=[0, 5])
    stats = serve.summarize(res, shots, 400.0)
    say(stats)
    assert np.all(np.isfinite(res["latency"])) and np.all(res["latency"] > 0)
    for i in (0, 5):
        assert np.array_equal(res["images"][i].cpu().numpy(),
                              xrt.simulate(shots[i], fh, precision="mixed").cpu().numpy())
    srv.close()


def heavy_small_shots(n, seed):
    """Small ROIs with many terms per pixel: their sums are split into parts
    (compute chunks, then reduce chunks on the server)."""
    base = synth.full_shot()
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        s = synth.served_shot(rng, base.F, base.hkl_min)
        w, h = int(rng.integers(16, 72)), int(rng.integers(16, 72))
        f0, s0 = int(rng.integers(900, 1500)), int(rng.integers(900, 1500))
        n_src, n_mos = int(rng.integers(30, 101)), int(rng.integers(8, 25))
        s = s.replace(roi=(f0, f0 + w, s0, s0 + h), src_dir=s.src_dir[:n_src].copy(),
                      src_lambda=s.src_lambda[:n_src].copy(),
                      src_weight=s.src_weight[:n_src] / s.src_weight[:n_src].sum(), umats=s.umats[:n_mos].copy())
        out.append(s)
    return base, out


def expected_split(shot):
    f0, f1, s0, s1 = shot.roi
    tiles = -(-(f1 - f0) // 16) * -(-(s1 - s0) // 16)
    n_outer = shot.oversample ** 2 * shot.n_layers * shot.n_src
    if tiles >= 2048:
        return 1
    return max(1, min(-(-2048 // tiles), n_outer, n_outer * shot.n_phi * shot.n_mos // 1024, 64))


def expected_segments(shot, segment_terms):
    """Segments of each unit's outer iterations (xrt_server_desc.segment_terms):
    the fewest that keep a unit's pixel-terms within the budget, at most the
    shortest part's outer iterations."""
    split = expected_split(shot)
    n_outer = shot.oversample ** 2 * shot.n_layers * shot.n_src
    per_unit = 256 * (shot.terms_per_pixel // split)
    return max(1, min(-(-per_unit // segment_terms), n_outer // split))


@pytest.mark.parametrize("precision,shape", [("mixed", synth.SHAPE_SINCG), ("fp64", synth.SHAPE_SINCG),
                                             ("mixed", synth.SHAPE_GAUSS), ("fp64", synth.SHAPE_GAUSS)])
def test_segmented_sums_bitwise(precision, shape):
    """Sums run as consecutive segments, each continuing the running sums the
    previous one left in the arena (a small segment budget forces many, on
    whole and on split sums): every image equals the standalone call's bit
    for bit, in the mix and alone."""
    seg_terms = 1 << 12
    base, light = small_served_shots(4, seed=91)
    _, heavy = heavy_small_shots(2, seed=94)
    shots = light + heavy
    if shape == synth.SHAPE_GAUSS:
        rng = np.random.default_rng(93)
        shots = [x.replace(shape=shape, N=rng.uniform(5.0, 40.0, 3)) for x in shots]
    segs = [expected_segments(x, seg_terms) for x in shots]
    splits = [expected_split(x) for x in shots]
    say("segments", segs, "splits", splits)
    assert min(segs) > 1 and any(k > 1 for k in splits)
    fh = xrt.Fhkl.from_shot(base)
    ref = [xrt.simulate(x, fh, precision=precision).cpu().numpy() for x in shots]
    srv = xrt.Server(fh, hbm_budget=256 << 20, precision=precision, shape=shape, segment_terms=seg_terms)
    tickets = [srv.submit(x) for x in shots]
    drain(srv, tickets)
    for i, t in enumerate(tickets):
        assert np.array_equal(srv.image(t).cpu().numpy(), ref[i]), f"shot {i} ({segs[i]} segments) differs in the mix"
        srv.release(t)
    t = srv.submit(shots[-1])
    drain(srv, [t])
    assert np.array_equal(srv.image(t).cpu().numpy(), ref[-1]), "split shot differs alone"
    srv.release(t)
    srv.close()


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_served_split_shots(precision):
    """Split shots (part sums in the arena, reduce chunks after every part is
    done) beside whole-sum shots: each image equals the standalone call's bit
    for bit, in the mix and alone; one split image against the oracle."""
    base, heavy = heavy_small_shots(4, seed=21)
    _, light = small_served_shots(4, seed=22, max_side=64)
    shots = [x for pair in zip(heavy, light) for x in pair]
    splits = [expected_split(s) for s in shots]
    say("split factors", splits)
    assert max(splits) > 1 and min(splits) == 1
    fh = xrt.Fhkl.from_shot(base)
    ref = [xrt.simulate(s, fh, precision=precision).cpu().numpy() for s in shots]
    srv = xrt.Server(fh, hbm_budget=256 << 20, precision=precision)
    tickets = [srv.submit(s) for s in shots]
    drain(srv, tickets)
    for i, t in enumerate(tickets):
        assert np.array_equal(srv.image(t).cpu().numpy(), ref[i]), f"shot {i} (split {splits[i]}) differs in the mix"
        srv.release(t)
    for i in (0, 2):
        t = srv.submit(shots[i])
        drain(srv, [t])
        assert np.array_equal(srv.image(t).cpu().numpy(), ref[i]), f"shot {i} differs alone"
        srv.release(t)
    srv.close()
    if precision == "mixed":
        r = compare(ref[0], o.simulate(shots[0]))
        say("split shot vs oracle", r)
        assert r["zeros_ok"] and r["max_rel"] <= 1e-5


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_served_clamped_shots(precision):
    """A small structure-factor table ([-20, 20]^3, F_default 3) under the
    full-size detector: regions near the detector edge reach |h| ~ 60, so those
    shots take the clamped table index (and the default value), the central
    ones the clamp-free index; each image equals the standalone call's bit for
    bit, in one mix."""
    tiny = synth.tiny_shot()
    base = synth.full_shot()
    rng = np.random.default_rng(31)
    shots = []
    for k in range(6):
        s = synth.served_shot(rng, tiny.F, tiny.hkl_min).replace(F_default=3.0)
        n_src, n_mos = int(rng.integers(2, 9)), int(rng.integers(2, 9))
        w = 48
        f0 = [0, 2463 - w, 1200, 0, 2463 - w, 1230][k]
        s0 = [0, 2527 - w, 1250, 2527 - w, 0, 1240][k]
        s = s.replace(roi=(f0, f0 + w, s0, s0 + w), src_dir=s.src_dir[:n_src].copy(),
                      src_lambda=s.src_lambda[:n_src].copy(),
                      src_weight=s.src_weight[:n_src] / s.src_weight[:n_src].sum(), umats=s.umats[:n_mos].copy())
        assert s.n_fast == base.n_fast and s.n_slow == base.n_slow
        shots.append(s)
    fh = xrt.Fhkl.from_shot(shots[0])
    ref = [xrt.simulate(s, fh, precision=precision).cpu().numpy() for s in shots]
    srv = xrt.Server(fh, hbm_budget=64 << 20, precision=precision)
    tickets = [srv.submit(s) for s in shots]
    drain(srv, tickets)
    for i, t in enumerate(tickets):
        assert np.array_equal(srv.image(t).cpu().numpy(), ref[i]), f"shot {i} differs"
        srv.release(t)
    srv.close()
    # the edge regions do reach outside the table: their default-valued terms
    # make them differ from a run with F_default = 0
    fh0 = xrt.Fhkl.from_shot(shots[0].replace(F_default=0.0))
    edge0 = xrt.simulate(shots[0], fh0, precision=precision).cpu().numpy()
    assert not np.array_equal(edge0, ref[0])


def test_cancel_queued_shots():
    """With room for one shot at a time, the queued shots behind the first can
    be withdrawn; an admitted one cannot; the rest still equal their
    standalone images."""
    base, shots = small_served_shots(5, seed=41, max_side=64)
    shots = [s.replace(roi=(100 + 9 * i, 100 + 9 * i + 400, 300, 300 + 400)) for i, s in enumerate(shots)]
    fh = xrt.Fhkl.from_shot(base)
    srv = xrt.Server(fh, hbm_budget=1 << 20, max_resident=1, precision="mixed")  # one 400 x 400 image fits
    tickets = [srv.submit(s) for s in shots]
    srv.progress()
    assert srv.info(tickets[0]).state == xrt.XRT_SHOT_RUNNING
    with pytest.raises(xrt.XrtError) as e:
        srv.cancel(tickets[0])
    assert e.value.code == xrt.XRT_EBUSY
    srv.cancel(tickets[1])
    srv.cancel(tickets[3])
    with pytest.raises(xrt.XrtError):
        srv.info(tickets[1])
    keep = [0, 2, 4]
    t0 = time.time()
    pending = [tickets[i] for i in keep]
    while pending:
        srv.progress()
        for t in list(pending):
            if srv.info(t).state == xrt.XRT_SHOT_DONE:
                i = tickets.index(t)
                assert np.array_equal(srv.image(t).cpu().numpy(),
                                      xrt.simulate(shots[i], fh, precision="mixed").cpu().numpy())
                srv.release(t)
                pending.remove(t)
        assert time.time() - t0 < 60
    srv.close()
