"""Throughput of the per-pixel X-ray tracing sum on one MI355X.

One step = one full-size shot: 2463 x 2527 pixels x 2^2 sub-pixels x 3 sensor
layers x 100 sources x 50 mosaic domains = 3.7344e11 pixel terms, binary64,
inputs (tables, structure factors) resident on the device; the step is the
xrt_simulate call (small table upload + the spots kernel).  The same shot is
also timed in the mixed-precision form and its error against the oracle on
sampled pixels is reported beside it; so is the background of a water-like
scatterer over the same detector.

Prints one JSON line.  Synthetic, seeded inputs (synth.full_shot).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic work of one pixel term of the method, frozen: floating-point
# operations the definition itself prescribes, independent of how a kernel
# implements them (each is derived in the design notes, "Roofline counts").
# An addition, subtraction or multiplication is 1 flop, a fused multiply-add
# 2, a division or square root 1; rint, compares, selects and the table
# gather are not flops.  A function without a hardware instruction of the
# required accuracy is priced as the minimax polynomial of the lowest degree
# that reaches it, by Horner's rule: sin(pi x) on |x| <= 1/2 as x P(x^2) with
# P of degree 7 for binary64 (16 flops), degree 4 for binary32 (10); exp on
# the reduced range |r| <= ln2/2 with a degree-11 polynomial after a
# Cody-Waite reduction for binary64 (27 flops); binary32 exp is the hardware
# exp2 after a multiplication by log2(e) (2 flops).
#   sincg, binary64: h = M S 15, f 3, g = N f - rint(N f) 6, six sines 96,
#     ratio and square 6, F^2 L^2 and the sum 2                      -> 128
#   sincg, mixed: binary64 h, f, g (24); binary32 six sines 60, ratio and
#     square 6, F^2 L^2 1, Kahan sum 4 (71)
#   Gaussian forward, binary64: h 15, f 3, exponent 9, exp 27, F^2 L^2 and
#     the sum 2                                                      -> 56
#   Gaussian forward, mixed: binary64 h, f, exponent and e - m (28); binary32
#     exp 2, F^2 exp 1, Kahan sum 4 (7)
#   adjoint, binary64: S' = Q^T S 15, h 15, f 3, exponent 9, exp 27, w F^2 exp
#     2, per axis dL/dh (2 products, 3 FMA) and dL/dN (product, FMA, FMA) 39,
#     dL/dscale 1                                                    -> 111
#   adjoint, mixed: binary64 S', h, f, exponent, e - m (43); binary32 exp 2,
#     w F^2 exp 2, derivatives 39, dL/dscale 1 (44)
#   background, binary64: d - dir 3, its square 5, root 1, stol 1, the
#     interpolation 3, F^2 1, Kahn factor (three dot products 15, 1 + c^2 2,
#     x^2 - y^2 3, K term 2, half 1) 23, w P F^2 and the sum 3         -> 40
#   background, mixed: the same in binary32 plus the Kahan sum's 3 more (43)
FLOPS = {
    "spots": {"fp64": {"f64": 128, "f32": 0}, "mixed": {"f64": 24, "f32": 71}},
    "gauss_fwd": {"fp64": {"f64": 56, "f32": 0}, "mixed": {"f64": 28, "f32": 7}},
    "adjoint": {"fp64": {"f64": 111, "f32": 0}, "mixed": {"f64": 43, "f32": 44}},
    "background": {"fp64": {"f64": 40, "f32": 0}, "mixed": {"f64": 0, "f32": 43}},
}
# MI355X vector peaks (FMA = 2 flops): 256 CUs x 4 SIMDs x 2.4 GHz x 32
# binary32 lanes (157.3 TFLOP/s) or 16 binary64 lanes (78.6 TFLOP/s) per cycle
PEAK = {"f64": 256 * 4 * 16 * 2 * 2.4e9, "f32": 256 * 4 * 32 * 2 * 2.4e9}
HBM_PEAK = 8.0e12


def roofline_of(flops, terms_per_s):
    """Achieved algorithmic TFLOP/s and the fraction of the vector roofline:
    the time the flops of one term need at the binary64 and binary32 peaks,
    times the terms per second (a mixed term is priced in both)."""
    t_term = sum(flops[k] / PEAK[k] for k in flops)
    total = sum(flops.values())
    return {"achieved": total * terms_per_s / 1e12, "peak": total / t_term / 1e12,
            "frac": terms_per_s * t_term, "flop_per_term": dict(flops)}


# Issue efficiency (not a roofline): the implemented instruction sequence of
# the binary64 and mixed sincg loops weighted by their measured issue cost on
# gfx950, in binary32-lane-op units (binary32 op 1, binary64 op or conversion
# 2, binary32 transcendental 4, binary64 reciprocal 8); it follows the
# kernel, so a loop issued without stalls sits near 1.  binary64 loop: 93
# binary64 operations and one reciprocal per term (194); mixed: 33 binary64
# operations and conversions, 48 binary32 operations and one binary32
# reciprocal (118).
ISSUE_SLOTS = {"fp64": 194, "mixed": 118}
ISSUE_PEAK = 256 * 4 * 32 * 2.4e9

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = [os.path.join(HERE, "paper_2205_07976_amd", "csrc", f)
                  for f in ("xrt_kernels.hip", "xrt_math.h", "xrt_internal.h")]


def kernel_src_sha():
    """sha256 (16 hex digits) of the device sources: the key that ties a
    committed counter summary to the kernels it measured."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fp:
            h.update(fp.read())
    return h.hexdigest()[:16]


def profile_keys(name):
    """The machine-readable figures of a committed counter summary under
    profiles/ (its '# bench-keys {json}' line), or None if the kernels have
    changed since its counters were taken or the file is missing."""
    path = os.path.join(HERE, "profiles", name)
    if not os.path.exists(path):
        return None
    with open(path) as fp:
        for line in fp:
            if line.startswith("# bench-keys "):
                keys = json.loads(line[len("# bench-keys "):])
                if keys.get("kernel_src_sha") == kernel_src_sha():
                    keys["source"] = f"profiles/{name}"
                    return keys
                return None
    return None


def read_sclk_mhz():
    """The shader clock of the first GPU that reports one, MHz (the active
    level of pp_dpm_sclk in sysfs), or None where sysfs does not expose it."""
    import glob
    import re
    for f in sorted(glob.glob("/sys/class/drm/card*/device/pp_dpm_sclk")):
        try:
            with open(f) as fp:
                for line in fp:
                    if "*" in line:
                        m = re.search(r"(\d+)\s*Mhz", line, re.I)
                        if m:
                            return float(m.group(1))
        except OSError:
            continue
    return None


class SclkSampler:
    """Samples read_sclk_mhz() every period_s in a thread while the timed
    region runs (a sysfs read: no GPU work)."""

    def __init__(self, period_s=0.05):
        import threading
        self.samples, self.period, self._stop = [], period_s, threading.Event()
        self._t = threading.Thread(target=self._run, daemon=True)

    def _run(self):
        while not self._stop.is_set():
            v = read_sclk_mhz()
            if v is not None:
                self.samples.append(v)
            self._stop.wait(self.period)

    def __enter__(self):
        self._t.start()
        return self

    def __exit__(self, *exc):
        self._stop.set()
        self._t.join()

    def summary(self):
        if not self.samples:
            return {"mhz_median": None, "note": "sysfs pp_dpm_sclk not readable on this host"}
        v = np.array(self.samples)
        return {"mhz_median": float(np.median(v)), "mhz_min": float(v.min()), "mhz_max": float(v.max()),
                "samples": len(v)}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_form(shot, fh, precision, steps, warmup):
    import torch
    from paper_2205_07976_amd import xrt
    out = torch.empty(shot.roi_shape, dtype=torch.float64 if precision == "fp64" else torch.float32,
                      device="cuda")
    for _ in range(warmup):
        xrt.simulate(shot, fh, precision=precision, out=out)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record()
        xrt.simulate(shot, fh, precision=precision, out=out)
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = [a.elapsed_time(b) for a, b in evs]
    return out, wall, ev_ms


def host_threads():
    """Host threads for the oracle: the CPUs this process may run on, capped
    by OMP_NUM_THREADS when it is set (the share of the host that goes with
    one GPU on a shared machine)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(n, 1)


def host_description():
    """What the CPU baseline ran on: the CPU model (lscpu), the logical CPUs
    of the host (os.cpu_count), the ones this process may use (affinity) and
    the cgroup CPU quota, if any."""
    model = ""
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    quota = None
    try:
        with open("/sys/fs/cgroup/cpu.max") as fp:
            q, per = fp.read().split()
            quota = None if q == "max" else float(q) / float(per)
    except Exception:
        pass
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None,
            "cgroup_cpu_quota": quota, "omp_num_threads_env": os.environ.get("OMP_NUM_THREADS")}


def cpu_baseline(shot, budget_s=15.0):
    """The oracle on a seeded pixel subset sized to about budget_s seconds,
    on every host thread this process may use."""
    import synth
    from oracle import oracle as o
    cores = host_threads()
    n = 64
    while True:
        pix = synth.pixel_sample(shot, n, 99)
        t0 = time.perf_counter()
        o.simulate(shot, pix, nthreads=cores)
        dt = time.perf_counter() - t0
        if dt >= 0.6 * budget_s or n >= 262144:
            break
        n = min(262144, max(2 * n, int(n * budget_s / max(dt, 1e-3))))
    terms = n * shot.terms_per_pixel
    rate = terms / dt / 1e9
    return {"value": rate, "unit": "Gterm/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} seeded pixels of the full-size shot ({terms:.3e} terms, {dt:.1f} s)",
            "per_core": rate / cores, "host": host_description(),
            "full_shot_s_extrapolated": shot.n_terms / (rate * 1e9)}


def background_bench(shot, steps):
    """The background of the water-like scatterer over the full-size detector
    (1200 terms per pixel: no spindle or mosaic loop), both precisions, timed
    with HIP events around each call on the current stream; a sampled check
    against the oracle; the oracle's own rate on a pixel subset."""
    import numpy as np
    import torch
    import synth
    from oracle import oracle as o
    from paper_2205_07976_amd import xrt
    bg = synth.water_background()
    terms = shot.n_pixels * shot.oversample ** 2 * shot.n_layers * shot.n_src
    out = {"workload": f"water-like curve ({bg.n_knots} knots) over the full-size detector: "
                       "2463x2527 px, oversample 2, 3 layers, 100 sources = 1200 terms/px",
           "terms": terms, "unit": "TFLOP/s"}
    pix = synth.pixel_sample(shot, 256, 77)
    ref = o.background(shot, bg, pix, nthreads=host_threads())
    n = max(steps, 5)
    for prec in ("fp64", "mixed"):
        img = torch.empty(shot.roi_shape, dtype=torch.float64 if prec == "fp64" else torch.float32, device="cuda")
        xrt.simulate_background(shot, bg, precision=prec, out=img)
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
        for a, b in evs:
            a.record()
            xrt.simulate_background(shot, bg, precision=prec, out=img)
            b.record()
        torch.cuda.synchronize()
        ms = sum(a.elapsed_time(b) for a, b in evs) / n
        x = img.cpu().numpy()[pix[:, 1], pix[:, 0]].astype(np.float64)
        rf = roofline_of(FLOPS["background"][prec], terms / (ms * 1e-3))
        out[prec] = {"ms": ms, "Gterm_s": terms / ms / 1e6, **rf,
                     "max_rel_err": float(np.max(np.abs(x - ref) / ref)), "err_sample": "256 seeded pixels"}
        log(f"background {prec}: {ms:.2f} ms, {terms / ms / 1e6:.0f} Gterm/s, frac {rf['frac']:.3f}")
    cores = host_threads()
    sample = synth.pixel_sample(shot, 262144, 78)
    t0 = time.perf_counter()
    o.background(shot, bg, sample, nthreads=cores)
    dt = time.perf_counter() - t0
    out["cpu_oracle"] = {"Gterm_s": len(sample) * 1200 / dt / 1e9, "cores": cores,
                         "sample": f"{len(sample)} seeded pixels ({dt:.2f} s)"}
    return out


def ensemble_bench(shot, steps, n_images=16):
    """The ensemble sum: n_images distinct binary32 full-detector images
    (together larger than the 256 MB last-level cache) added one after another
    into one binary64 accumulator with xrt_add_image; per call 20 algorithmic
    bytes per pixel (4 read from the image, 8 read and 8 written in the
    accumulator) against the 8 TB/s HBM peak."""
    import numpy as np
    import torch
    from oracle import ensemble as ens
    from paper_2205_07976_amd import xrt
    ns, nf = shot.n_slow, shot.n_fast
    gen = torch.Generator(device="cuda")
    gen.manual_seed(12)
    imgs = [torch.rand((ns, nf), generator=gen, device="cuda", dtype=torch.float32) for _ in range(n_images)]
    acc = torch.zeros((ns, nf), dtype=torch.float64, device="cuda")
    for im in imgs[:2]:
        xrt.add_image(acc, im)
    torch.cuda.synchronize()
    n = max(steps, 3)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    for a, b in evs:
        a.record()
        for im in imgs:
            xrt.add_image(acc, im)
        b.record()
    torch.cuda.synchronize()
    ms = sum(a.elapsed_time(b) for a, b in evs) / n / n_images
    bytes_call = 20.0 * ns * nf
    gbs = bytes_call / (ms * 1e-3) / 1e9
    # parity on a corner block: the accumulator holds 2 + n * n_images adds
    blk = (slice(0, 64), slice(0, 64))
    ref = np.zeros((64, 64))
    for im in imgs[:2] + imgs * n:
        ref = ens.add_image(ref, im[blk].cpu().numpy(), 0, 0)
    exact = bool(np.array_equal(acc[blk].cpu().numpy(), ref))
    log(f"ensemble add: {ms * 1e3:.1f} us per full-detector image, {gbs:.0f} GB/s ({gbs / 8000:.3f} of HBM peak)")
    # the same images in one xrt_add_images call: the accumulator is read and
    # written once for the batch (4 + 16 / n_images algorithmic bytes per
    # pixel and image)
    xrt.add_images(acc, imgs)
    torch.cuda.synchronize()
    evb = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    for a, b in evb:
        a.record()
        xrt.add_images(acc, imgs)
        b.record()
    torch.cuda.synchronize()
    msb = sum(a.elapsed_time(b) for a, b in evb) / n / n_images
    gbsb = (4.0 + 16.0 / n_images) * ns * nf / (msb * 1e-3) / 1e9
    log(f"ensemble add, one call for {n_images} images: {msb * 1e3:.1f} us per image, {gbsb:.0f} GB/s")
    return {"workload": f"{n_images} distinct binary32 2463x2527 images added in turn into one binary64 accumulator",
            "us_per_image": ms * 1e3, "bytes_per_call": bytes_call,
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": 8000.0, "unit": "GB/s", "frac": gbs / 8000.0},
            "corner_block_bitwise_equal_oracle": exact,
            "batched": {"us_per_image": msb * 1e3, "bytes_per_image": (4.0 + 16.0 / n_images) * ns * nf,
                        "achieved_GBs": gbsb, "frac": gbsb / 8000.0}}


def image_error(shot, img):
    """Max and RMS relative error of an image of the full shot against the
    oracle on 256 seeded pixels (the same pixels for every image)."""
    import numpy as np
    import synth
    from oracle import oracle as o
    pix = synth.pixel_sample(shot, 256, 2024)
    ref = o.simulate(shot, pix, nthreads=host_threads())
    x = img[pix[:, 1], pix[:, 0]].astype(np.float64)
    r = np.abs(x - ref) / ref
    return float(r.max()), float(np.sqrt(np.mean(r * r)))


def adjoint_bench(steps):
    """The refinement workload: 512 regions of 32 x 32 pixels around predicted
    spots of the full-size crystal with the Gaussian shape (60000 terms per
    pixel); squared-residual loss against a target simulated at perturbed
    parameters with Poisson noise; forward (regions) + adjoint per step."""
    import math
    import numpy as np
    import torch
    import synth
    from paper_2205_07976_amd import refine, xrt
    shot, origins = synth.roi_shot()
    fh = xrt.Fhkl.from_shot(shot)
    size = (32, 32)
    abc_t, beta_t, N_t, th_t, s_t = refine.perturbed(np.array([79.0, 79.0, 38.0]), math.radians(95.0),
                                                     shot.N, 1.0)
    Mt = refine.m0_from_params(torch.tensor(abc_t), torch.tensor(beta_t), torch.tensor(th_t), shot.U).numpy()
    clean = xrt.simulate_rois(shot.replace(U=np.eye(3), cell=Mt, N=N_t, scale=s_t), fh, origins, size)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    k = 1e4 / float(clean.max())
    target = torch.poisson(clean * k, generator=gen) / k
    base = shot.replace(U=np.eye(3), cell=(shot.U @ shot.cell.T).T.copy())
    terms = len(origins) * size[0] * size[1] * shot.terms_per_pixel
    out = {"workload": "512 ROIs of 32x32 px around predicted spots, Gaussian N=20, 60000 terms/px",
           "terms_per_pass": terms}
    grads = {}
    for prec in ("fp64", "mixed"):
        img = xrt.simulate_rois(base, fh, origins, size, precision=prec, out_dtype=torch.float64)
        g = xrt.backward_rois(base, fh, origins, size, 2 * (img - target), precision=prec)
        torch.cuda.synchronize()
        ef = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        eb = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        for (a, b), (c, d) in zip(ef, eb):
            a.record()
            xrt.simulate_rois(base, fh, origins, size, precision=prec, out=img)
            b.record()
            r = 2 * (img - target)
            c.record()
            xrt.backward_rois(base, fh, origins, size, r, precision=prec, grad=g)
            d.record()
        torch.cuda.synchronize()
        fms = sum(a.elapsed_time(b) for a, b in ef) / steps
        bms = sum(c.elapsed_time(d) for c, d in eb) / steps
        grads[prec] = g.cpu().numpy()
        out[prec] = {"fwd_ms": fms, "bwd_ms": bms, "fwd_Gterm_s": terms / fms / 1e6,
                     "bwd_Gterm_s": terms / bms / 1e6,
                     "fwd_roofline": roofline_of(FLOPS["gauss_fwd"][prec], terms / (fms * 1e-3)),
                     "bwd_roofline": roofline_of(FLOPS["adjoint"][prec], terms / (bms * 1e-3)),
                     "loss": float(((img - target) ** 2).sum())}
        log(f"adjoint {prec}: forward {fms:.1f} ms (frac {out[prec]['fwd_roofline']['frac']:.3f}), "
            f"backward {bms:.1f} ms (frac {out[prec]['bwd_roofline']['frac']:.3f})")
    # the oracle's binary64 gradient on a seeded sample of the regions'
    # pixels (dL/dI of the binary64 residual), on every host thread
    from oracle import oracle as o
    rng = np.random.default_rng(55)
    pick = rng.choice(len(origins) * size[0] * size[1], 1024, replace=False)
    q, rem = np.divmod(pick, size[0] * size[1])
    ls, lf = np.divmod(rem, size[0])  # [n_roi][ns][nf], size = (nf, ns)
    pix = np.stack([origins[q, 0] + lf, origins[q, 1] + ls], axis=1).astype(np.int32)
    img64 = xrt.simulate_rois(base, fh, origins, size, precision="fp64", out_dtype=torch.float64)
    res = (2 * (img64 - target)).cpu().numpy().reshape(-1)[pick]
    cores = host_threads()
    t0 = time.perf_counter()
    o.gradient(base, pix, res, nthreads=cores)
    dt = time.perf_counter() - t0
    out["cpu_oracle_gradient"] = {"Gterm_s": len(pix) * shot.terms_per_pixel / dt / 1e9, "cores": cores,
                                  "sample": f"{len(pix)} seeded pixels of the 512 regions ({dt:.2f} s)"}
    log(f"adjoint: oracle gradient {out['cpu_oracle_gradient']}")
    d = np.abs(grads["mixed"] - grads["fp64"])
    out["grad_fp64"] = grads["fp64"].tolist()
    out["mixed_vs_fp64_max_diff_over_max"] = [float(d[sl].max() / np.abs(grads["fp64"][sl]).max())
                                              for sl in (slice(0, 9), slice(9, 12), slice(12, 13))]
    return out


def standalone_times(shots, fh, precision, tag):
    """Each shot's time as one standalone xrt_simulate call (HIP events on the
    launch stream around the call), one call per shot after one warm-up; the
    images go to one reused buffer."""
    import torch
    from paper_2205_07976_amd import xrt
    dt = torch.float64 if precision == "fp64" else torch.float32
    buf = torch.empty(max(s.n_pixels for s in shots), dtype=dt, device="cuda")
    xrt.simulate(shots[0], fh, precision=precision, out=buf[:shots[0].n_pixels].view(shots[0].roi_shape))
    torch.cuda.synchronize()
    out = np.empty(len(shots))
    batch = 100
    for b0 in range(0, len(shots), batch):
        evs = []
        for s in shots[b0:b0 + batch]:
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            xrt.simulate(s, fh, precision=precision, out=buf[:s.n_pixels].view(s.roi_shape))
            b.record()
            evs.append((a, b))
        torch.cuda.synchronize()
        out[b0:b0 + len(evs)] = [a.elapsed_time(b) * 1e-3 for a, b in evs]
        log(f"  standalone {tag}: {b0 + len(evs)}/{len(shots)} shots timed")
    return out


def latency_stats(res, shots, t_alone, offered_rate=None):
    """serve.summarize plus the slowdown: each shot's latency over its own
    standalone time (1 = served as fast as alone on an idle device)."""
    from paper_2205_07976_amd import serve
    out = serve.summarize(res, shots, offered_rate)
    slow = res["latency"] / t_alone
    out["p50_slowdown"] = float(np.percentile(slow, 50))
    out["p99_slowdown"] = float(np.percentile(slow, 99))
    out["mean_slowdown"] = float(np.mean(slow))
    return out


def serving_bench(n_pool=1000, n_cap=200, n_fp64=60, loads=(0.5, 0.8, 0.95), policy="shortest_remaining"):
    """The served shot stream (independent shots: random orientation,
    log-uniform ROI 64..2463 x 64..2527 px, 1-100 sources, 1-200 domains,
    N in [5, 40], the full-size detector and shared table).  A pool of n_pool
    shots is timed standalone first (mixed); n_cap of them submitted at once
    give the capacity; then all n_pool arrive as a Poisson stream at each
    load x capacity (a seeded order per load).  Latency is submit -> result
    ready on the server's clock; slowdown is latency over the shot's
    standalone time; the offered rate of a load is load x the capacity in
    terms/s over the pool's mean terms per shot.  Also: the capacity of a binary64 server against the
    binary64 standalone calls of the same shots, the capacity again under a
    256 MiB HBM budget, and the mixed capacity with the water-like background
    added to every image."""
    import synth
    from paper_2205_07976_amd import serve, xrt
    base = synth.full_shot()
    fh = xrt.Fhkl.from_shot(base)
    rng = np.random.default_rng(4)
    pool = [synth.served_shot(rng, base.F, base.hkl_min) for _ in range(n_pool)]
    terms = np.array([float(s.n_terms) for s in pool])
    log(f"serving: pool of {n_pool} shots, {terms.sum():.3e} terms (mean {terms.mean():.3e})")
    t_mixed = standalone_times(pool, fh, "mixed", "mixed")

    def progress(tag, n):
        def cb(i, t, count=[0]):
            count[0] += 1
            if count[0] % 100 == 0 or count[0] == n:
                log(f"  {tag}: {count[0]}/{n} shots done")
        return cb

    out = {"workload": "served stream: log-uniform ROI, 1-100 sources, 1-200 domains, N in [5,40], "
                       "full-size detector and table, mixed",
           "policy": policy,
           "pool": {"shots": n_pool, "terms": float(terms.sum()),
                    "standalone_mixed_s": float(t_mixed.sum()),
                    "standalone_mixed_Gterm_s": float(terms.sum() / t_mixed.sum() / 1e9)}}
    srv = xrt.Server(fh, hbm_budget=16 << 30, max_resident=64, precision="mixed", policy=policy)
    serve.run_stream(srv, pool[:2], np.zeros(2))  # the persistent kernel's first launch
    cap = pool[:n_cap]
    res = serve.run_stream(srv, cap, np.zeros(n_cap), on_done=progress("capacity", n_cap))
    closed = latency_stats(res, cap, t_mixed[:n_cap])
    closed["standalone_s"] = float(t_mixed[:n_cap].sum())
    closed["vs_standalone"] = closed["standalone_s"] / closed["makespan_s"]
    out["closed_loop"] = closed
    log(f"serving: capacity {closed['images_per_s']:.2f} img/s, {closed['Gterm_per_s']:.0f} Gterm/s, "
        f"{closed['vs_standalone']:.3f} of the standalone calls")
    # offered load in work: shots of the whole pool arrive at `load` times
    # the capacity in terms/s over the pool's mean shot (the 200-shot subset's
    # image rate would misstate it, its mean shot differing from the pool's)
    mean_terms = float(terms.mean())
    out["pool"]["mean_terms"] = mean_terms
    for load in loads:
        order = np.random.default_rng(int(round(load * 100))).permutation(n_pool)
        shots = [pool[i] for i in order]
        rate = load * closed["Gterm_per_s"] * 1e9 / mean_terms
        arr = serve.poisson_arrivals(np.random.default_rng(int(round(load * 1000))), n_pool, rate)
        res = serve.run_stream(srv, shots, arr, on_done=progress(f"load {load:.2f}", n_pool), timeout=900.0)
        st = latency_stats(res, shots, t_mixed[order], rate)
        st["load"] = load
        st["offered_Gterm_per_s"] = rate * mean_terms / 1e9
        out[f"poisson_{load:.2f}"] = st
        log(f"serving at {load:.2f} x capacity: p50 {st['p50_ms']:.1f} ms, p99 {st['p99_ms']:.1f} ms, "
            f"slowdown p50 {st['p50_slowdown']:.2f} p99 {st['p99_slowdown']:.2f}, {st['Gterm_per_s']:.0f} Gterm/s")
    srv.close()
    # admission under a small HBM budget: the capacity run again with 256 MiB
    # (fewer shots resident at once; the largest image is 25 MB)
    srv = xrt.Server(fh, hbm_budget=256 << 20, max_resident=64, precision="mixed", policy=policy)
    serve.run_stream(srv, pool[:2], np.zeros(2))
    small = serve.summarize(serve.run_stream(srv, cap, np.zeros(n_cap)), cap)
    srv.close()
    small["vs_standalone"] = closed["standalone_s"] / small["makespan_s"]
    out["closed_loop_256MiB"] = small
    log(f"serving under a 256 MiB budget: {small['images_per_s']:.2f} img/s ({small['vs_standalone']:.3f})")
    # binary64: served capacity against standalone binary64 calls
    sub = pool[:n_fp64]
    t64 = standalone_times(sub, fh, "fp64", "fp64")
    srv = xrt.Server(fh, hbm_budget=16 << 30, max_resident=64, precision="fp64", policy=policy)
    serve.run_stream(srv, sub[:2], np.zeros(2))
    c64 = serve.summarize(serve.run_stream(srv, sub, np.zeros(n_fp64)), sub)
    srv.close()
    c64["standalone_s"] = float(t64.sum())
    c64["standalone_Gterm_s"] = float(terms[:n_fp64].sum() / t64.sum() / 1e9)
    c64["vs_standalone"] = c64["standalone_s"] / c64["makespan_s"]
    out["closed_loop_fp64"] = c64
    log(f"serving binary64: {c64['Gterm_per_s']:.0f} Gterm/s served, {c64['standalone_Gterm_s']:.0f} standalone "
        f"({c64['vs_standalone']:.3f})")
    # the mixed closed loop with the water-like background on every image
    srv = xrt.Server(fh, hbm_budget=16 << 30, max_resident=64, precision="mixed",
                     background=synth.water_background(), policy=policy)
    serve.run_stream(srv, sub[:2], np.zeros(2))
    out["closed_loop_with_background"] = serve.summarize(serve.run_stream(srv, sub, np.zeros(n_fp64)), sub)
    srv.close()
    log(f"serving with the background: {out['closed_loop_with_background']['images_per_s']:.2f} img/s")
    return out


def serving_io_bench(n_shots=40, write_ms=20.0, writers=4, budgets=(256 << 20, 64 << 20)):
    """The served stream with every image written out by the client: each
    image is written to a file and the writer then waits write_ms more (a
    slow remote filesystem), under HBM budgets of 256 and 64 MiB.  A client that
    copies each image from the device and writes it in its loop, against a
    write-out server (images copied to pinned host memory on a copy stream,
    device memory freed at once) with `writers` writer threads; and, between
    the two, the in-place server with writer threads."""
    import shutil
    import tempfile
    import numpy as np
    import synth
    from paper_2205_07976_amd import serve, xrt
    base = synth.full_shot()
    fh = xrt.Fhkl.from_shot(base)
    rng = np.random.default_rng(31)
    shots = [synth.served_shot(rng, base.F, base.hkl_min) for _ in range(n_shots)]
    d = tempfile.mkdtemp(prefix="xrt_io_")
    out = {"workload": f"{n_shots} served shots at once, mixed; every image written to a "
                       f"file, then {write_ms:g} ms more per image"}

    def sink(i, img):
        path = os.path.join(d, f"img{i}.bin")
        img.tofile(path)
        os.remove(path)
        time.sleep(write_ms * 1e-3)

    try:
        for budget in budgets:
            for name, host_budget, nw in (("in_place_loop", 0, 0), ("in_place_threads", 0, writers),
                                          ("write_out_threads", 2 << 30, writers)):
                srv = xrt.Server(fh, hbm_budget=budget, max_resident=64, precision="mixed", host_budget=host_budget)
                serve.run_stream(srv, shots[:2], np.zeros(2), sink=sink, writers=nw)
                r = serve.summarize(serve.run_stream(srv, shots, np.zeros(n_shots), sink=sink, writers=nw), shots)
                srv.close()
                key = f"budget_{budget >> 20}MiB"
                out.setdefault(key, {})[name] = r
                log(f"serving with images written out, {key} {name}: {r['images_per_s']:.2f} img/s, "
                    f"p50 {r['p50_ms']:.0f} ms")
    finally:
        shutil.rmtree(d, ignore_errors=True)
    return out


def served_region_bench(steps, side=1024):
    """One side x side region of the full-size shot served alone (the only
    shot on the server, so the persistent kernel runs its chunks and nothing
    else) against the standalone call on the same region, both precisions:
    the per-term cost of the served kernel, free of the stream's mix."""
    import torch
    import synth
    from paper_2205_07976_amd import serve, xrt
    shot = synth.full_shot()
    fh = xrt.Fhkl.from_shot(shot)
    f0, s0 = 1231 - side // 2, 1263 - side // 2
    reg = shot.replace(roi=(f0, f0 + side, s0, s0 + side))
    out = {"workload": f"{side}x{side} region of the full-size shot ({reg.n_terms:.3e} terms)"}
    n = max(steps, 3)
    for prec in ("fp64", "mixed"):
        _, _, ev = time_form(reg, fh, prec, n, 1)
        alone = sum(ev) / len(ev) * 1e-3
        srv = xrt.Server(fh, hbm_budget=1 << 30, max_resident=4, precision=prec)
        serve.run_stream(srv, [reg], np.zeros(1))
        lat = []
        for _ in range(n):
            r = serve.run_stream(srv, [reg], np.zeros(1))
            lat.append(float(r["latency"][0]))
        srv.close()
        torch.cuda.synchronize()
        served = float(np.median(lat))
        out[prec] = {"standalone_ms": alone * 1e3, "served_ms": served * 1e3, "served_vs_standalone": alone / served}
        log(f"served region {side}^2 {prec}: standalone {alone * 1e3:.1f} ms, served {served * 1e3:.1f} ms "
            f"({alone / served:.3f})")
    return out


SECTIONS = ("mixed", "small_roi", "background", "ensemble", "adjoint", "served_region", "serving", "serving_io", "cpu")
DEFAULT_SECTIONS = ("mixed", "small_roi", "background", "ensemble", "adjoint", "served_region", "serving", "cpu")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--only", default="",
                    help="comma-separated sections to run after the binary64 full shot (default: "
                         + ",".join(DEFAULT_SECTIONS) + "; also available: serving_io)")
    ap.add_argument("--serve-policy", default="shortest_remaining", choices=("shortest_remaining", "fair_share"),
                    help="publication order of the served stream's chunks")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="finish with one device-to-device copy of this many MiB (a kernel of known "
                         "traffic that calibrates the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); shots would be sharded "
              "one per GPU with no exchange, and no multi-GPU launch is provided.", file=sys.stderr)
        return 2
    sections = set(args.only.split(",")) - {""} if args.only else set(DEFAULT_SECTIONS)
    unknown = sections - set(SECTIONS)
    if unknown:
        print(f"unknown sections {sorted(unknown)}; choose from {SECTIONS}", file=sys.stderr)
        return 2

    import torch
    import synth
    from paper_2205_07976_amd import xrt

    torch.cuda.set_device(0)
    shot = synth.full_shot()
    fh = xrt.Fhkl.from_shot(shot)
    terms = shot.n_terms
    log(f"full-size shot: {terms:.4e} terms; fp64 warmup {args.warmup} steps {args.steps}")

    with SclkSampler() as sclk:
        img64, wall, ev = time_form(shot, fh, "fp64", args.steps, args.warmup)
    ms = 1e3 * wall / args.steps
    kern_ms = sum(ev) / len(ev)
    value = terms / (wall / args.steps) / 1e9
    rf = roofline_of(FLOPS["spots"]["fp64"], terms / (kern_ms * 1e-3))
    ctr = profile_keys("spots_full_shot_counters.txt")
    res = {
        "metric": "pixel-term evaluations/s (G/s) vs FP32 VALU peak; p50/p99 shot latency",
        "value": value, "unit": "Gterm/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "full-size shot, binary64: 2463x2527 px, oversample 2, 3 layers, "
                               "100 sources, 50 mosaic domains, sincg N=20, Fhkl [-60,60]^3",
                   "pixels": shot.n_pixels, "terms_per_pixel": shot.terms_per_pixel, "terms": terms},
        "roofline": {"bound": "alu", "achieved": rf["achieved"], "peak": rf["peak"], "unit": "TFLOP/s",
                     "frac": rf["frac"], "traffic": ctr["fp64"]["traffic_bytes"] if ctr else None,
                     "kernel": "spots_kernel<FP64,SINCG>", "kernel_ms": kern_ms,
                     "flop_per_term": rf["flop_per_term"],
                     "counters": ctr["fp64"] if ctr else None,
                     "counters_source": ctr["source"] if ctr else None,
                     "issue_efficiency": ISSUE_SLOTS["fp64"] * terms / (kern_ms * 1e-3) / ISSUE_PEAK,
                     "sclk_during_timed_region": sclk.summary()},
    }
    e64, r64 = image_error(shot, img64.cpu().numpy())
    res["max_rel_err"], res["rms_rel_err"] = e64, r64
    res["err_sample"] = "256 seeded pixels of the timed image against the oracle"
    log(f"fp64: {ms:.1f} ms/step (events {kern_ms:.1f} ms), {value:.1f} Gterm/s, "
        f"{rf['achieved']:.1f} algorithmic TFLOP/s, roofline frac {rf['frac']:.3f}, max rel err {e64:.2e}")

    if "mixed" in sections:
        img32, wall32, ev32 = time_form(shot, fh, "mixed", args.steps, args.warmup)
        k32 = sum(ev32) / len(ev32)
        v32 = terms / (wall32 / args.steps) / 1e9
        rf32 = roofline_of(FLOPS["spots"]["mixed"], terms / (k32 * 1e-3))
        emax, erms = image_error(shot, img32.cpu().numpy())
        res["mixed"] = {"value": v32, "unit": "Gterm/s", "ms_per_step": 1e3 * wall32 / args.steps,
                        "kernel_ms": k32, "roofline": rf32,
                        "counters": ctr["mixed"] if ctr else None,
                        "issue_efficiency": ISSUE_SLOTS["mixed"] * terms / (k32 * 1e-3) / ISSUE_PEAK,
                        "speedup_vs_fp64": v32 / value,
                        "max_rel_err": emax, "rms_rel_err": erms, "err_sample": "256 seeded pixels"}
        log(f"mixed: {1e3 * wall32 / args.steps:.1f} ms/step, {v32:.1f} Gterm/s, frac {rf32['frac']:.3f}, "
            f"max rel err {emax:.2e}")

    if "small_roi" in sections:
        # a small region of the same shot: its sums are split over many
        # workgroups (a 64 x 64 region is only 16 tiles)
        small = shot.replace(roi=(1200, 1264, 1250, 1314))
        res["small_roi"] = {"workload": "64x64 region of the full-size shot (2.46e8 terms, split sums)"}
        for prec in ("fp64", "mixed"):
            _, wall_s, ev_s = time_form(small, fh, prec, max(args.steps, 5), 1)
            ms_s = sum(ev_s) / len(ev_s)
            res["small_roi"][prec] = {"ms": ms_s, "Gterm_s": small.n_terms / ms_s / 1e6}
            log(f"small ROI {prec}: {ms_s:.2f} ms, {small.n_terms / ms_s / 1e6:.0f} Gterm/s")

    if "background" in sections:
        res["background"] = background_bench(shot, args.steps)
        res["background"]["image_fp64_ms"] = kern_ms + res["background"]["fp64"]["ms"]
        bgc = profile_keys("background_full_detector_counters.txt")
        res["background"]["counters"] = bgc
    if "ensemble" in sections:
        res["ensemble"] = ensemble_bench(shot, args.steps)
        res["ensemble"]["counters"] = profile_keys("ensemble_full_detector_counters.txt")
    if "adjoint" in sections:
        res["adjoint"] = adjoint_bench(args.steps)
        res["adjoint"]["counters"] = profile_keys("grad_rois_counters.txt")
    if "served_region" in sections:
        res["served_region"] = served_region_bench(args.steps)
        res["served_region"]["counters"] = profile_keys("serve_region_counters.txt")
    if "serving" in sections:
        res["serving"] = serving_bench(policy=args.serve_policy)
        res["p50_shot_latency_ms"] = res["serving"]["poisson_0.80"]["p50_ms"]
        res["p99_shot_latency_ms"] = res["serving"]["poisson_0.80"]["p99_ms"]
    if "serving_io" in sections:
        res["serving_io"] = serving_io_bench()

    if args.copy_mib:
        n = args.copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_mib} MiB read + {args.copy_mib} MiB written")

    if "cpu" in sections:
        res["cpu_baseline"] = cpu_baseline(shot)
        log(f"cpu oracle: {res['cpu_baseline']}")
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
