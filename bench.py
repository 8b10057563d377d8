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

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic VALU work of one pixel term (sincg inner loop), in FP32-lane-op
# equivalents: a binary32 or 32-bit integer op counts 1, a binary64 op or a
# conversion from binary64 counts 2 (binary64 runs at half the binary32 rate),
# a binary32 transcendental counts 4 (quarter rate), a binary64 reciprocal 8.
#   binary64: h = M S 12 ops; per axis 24 ops (rint, sub, max, N*f, rint, sub,
#             two squares, 2 x 7 FMA Horner, two products); 4 products;
#             reciprocal, one Newton step and a residual correction (rcp + 5);
#             square and FMA accumulate 2; table offset 3 FMA
#             -> 24 + 144 + 8 + 18 + 4 + 6 = 204
#   mixed:    h 12 binary64 ops; per axis 6 binary64 ops, 2 conversions and 12
#             binary32 ops; 4 products; rcp + mul; square and F^2 product;
#             Kahan 4; table offset 3 binary64 FMA
#             -> 24 + 84 + 4 + 5 + 2 + 4 + 6 = 129
C_ALG = {"fp64": 204, "mixed": 129}
# The background of an amorphous scatterer, per (pixel, sub-pixel, layer,
# source) term, same units:
#   binary64: d - dir 3 subs, |d - dir|^2 3 ops, its root (reciprocal square
#             root 8 + 5 ops), times 1/(2 lambda) 1, clamp to the first knot 1,
#             interval test 2 compares, interpolation 2, F^2 1, Kahn factor
#             (3 dot products 9 + 5), w P 1, accumulate 1
#             -> 6 + 6 + 18 + 2 + 2 + 4 + 4 + 2 + 28 + 4 = 76
#   mixed:    binary32 throughout: d - dir from heads and tails 9, square 3,
#             root 4, scale 1, clamp 1, compares 2, interpolation 2, F^2 1,
#             Kahn factor 14, products 2, Kahan add 4
#             -> 9 + 3 + 4 + 1 + 1 + 2 + 2 + 1 + 14 + 2 + 4 = 43
C_ALG_BG = {"fp64": 76, "mixed": 43}
# The refinement step (Gaussian shape), per pixel term, same units:
#   forward binary64: h 12 ops, per axis rint, sub, square, FMA (12 ops), exp
#             (clamp, scale, rint, 2 reduction FMAs, 11 Horner FMAs, ldexp,
#             conversion: 18 ops), table offset 3 FMAs, F^2 L^2 and the
#             accumulate 2 -> 24 + 24 + 36 + 6 + 4 = 94
#   forward mixed: h 12 and the axes 12 binary64 ops (48), exponent add and
#             conversion 4, binary32 exp 5, table offset 6, product 1, Kahan 4
#             -> 48 + 4 + 5 + 6 + 1 + 4 = 68
#   adjoint binary64: S' = Q^T S 9 ops, h 9, axes 12, table offset 3, exp 18,
#             two products, per axis the h derivative (2 products, 3 FMAs) and
#             the N derivative (product, 2 FMAs), dL/dscale 1
#             -> 18 + 18 + 24 + 6 + 36 + 4 + 48 + 2 = 156
#   adjoint mixed: S' 9 binary64 ops and 3 conversions (24), h 9 binary64 (18),
#             per axis rint and sub in binary64, a conversion, square and FMA
#             (24), table offset 6, binary32 exp and 2 products 7, derivatives
#             24 binary32 ops, dL/dscale 1 -> 24 + 18 + 24 + 6 + 7 + 24 + 1 = 104
C_ALG_REFINE = {"fwd": {"fp64": 94, "mixed": 68}, "bwd": {"fp64": 156, "mixed": 104}}
# MI355X binary32 VALU peak: 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz
# = 78.64 T lane-op/s (157.3 TFLOP/s counting an FMA as 2 flops)
PEAK_OPS = 256 * 4 * 32 * 2.4e9
# HBM bytes per binary64 launch from the FETCH_SIZE / WRITE_SIZE counters,
# each scaled by what it reads for a 1 GiB device copy (profiles/
# spots_full_shot_counters.txt); set to None whenever the kernel changes.
TRAFFIC_FP64 = 51.29e6


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


def cpu_baseline(shot, budget_s=15.0):
    """The oracle on a seeded pixel subset sized to about budget_s seconds."""
    import synth
    from oracle import oracle as o
    cores = min(16, os.cpu_count() or 1)
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
    return {"value": terms / dt / 1e9, "unit": "Gterm/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} seeded pixels of the full-size shot ({terms:.3e} terms, {dt:.1f} s)"}


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
           "terms": terms, "c_alg_per_term": C_ALG_BG, "peak": PEAK_OPS / 1e12,
           "unit": "T fp32-lane-op/s"}
    pix = synth.pixel_sample(shot, 256, 77)
    ref = o.background(shot, bg, pix, nthreads=min(16, os.cpu_count() or 1))
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
        ach = C_ALG_BG[prec] * terms / (ms * 1e-3)
        out[prec] = {"ms": ms, "Gterm_s": terms / ms / 1e6, "achieved": ach / 1e12, "frac": ach / PEAK_OPS,
                     "max_rel_err": float(np.max(np.abs(x - ref) / ref)), "err_sample": "256 seeded pixels"}
        log(f"background {prec}: {ms:.2f} ms, {terms / ms / 1e6:.0f} Gterm/s, frac {ach / PEAK_OPS:.3f}")
    cores = min(16, os.cpu_count() or 1)
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


def mixed_error(shot, img32):
    import numpy as np
    import synth
    from oracle import oracle as o
    pix = synth.pixel_sample(shot, 256, 2024)
    ref = o.simulate(shot, pix, nthreads=min(16, os.cpu_count() or 1))
    x = img32[pix[:, 1], pix[:, 0]].astype(np.float64)
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
           "terms_per_pass": terms, "c_alg_per_term": C_ALG_REFINE}
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
                     "fwd_frac": C_ALG_REFINE["fwd"][prec] * terms / (fms * 1e-3) / PEAK_OPS,
                     "bwd_frac": C_ALG_REFINE["bwd"][prec] * terms / (bms * 1e-3) / PEAK_OPS,
                     "loss": float(((img - target) ** 2).sum())}
        log(f"adjoint {prec}: forward {fms:.1f} ms (frac {out[prec]['fwd_frac']:.3f}), "
            f"backward {bms:.1f} ms (frac {out[prec]['bwd_frac']:.3f})")
    d = np.abs(grads["mixed"] - grads["fp64"])
    out["grad_fp64"] = grads["fp64"].tolist()
    out["mixed_vs_fp64_max_diff_over_max"] = [float(d[sl].max() / np.abs(grads["fp64"][sl]).max())
                                              for sl in (slice(0, 9), slice(9, 12), slice(12, 13))]
    return out


def serving_bench(n_cap=60, n_open=150, load=0.8):
    """The served shot stream: independent shots with a random orientation,
    log-uniform ROI (64..2463 x 64..2527 px), 1-100 sources, 1-200 domains,
    N in [5, 40], the full-size detector and shared table, mixed precision.
    Closed loop (all submitted at once) gives the capacity; then Poisson
    arrivals at `load` x capacity give the latency percentiles."""
    import numpy as np
    import synth
    from paper_2205_07976_amd import serve, xrt
    base = synth.full_shot()
    fh = xrt.Fhkl.from_shot(base)
    rng = np.random.default_rng(4)
    cap_shots = [synth.served_shot(rng, base.F, base.hkl_min) for _ in range(n_cap)]
    open_shots = [synth.served_shot(rng, base.F, base.hkl_min) for _ in range(n_open)]
    srv = xrt.Server(fh, hbm_budget=16 << 30, max_resident=64, precision="mixed")
    # warm-up: the persistent kernel's first launch
    serve.run_stream(srv, cap_shots[:2], np.zeros(2))
    closed = serve.summarize(serve.run_stream(srv, cap_shots, np.zeros(n_cap)), cap_shots)
    rate = load * closed["images_per_s"]
    arr = serve.poisson_arrivals(np.random.default_rng(6), n_open, rate)
    opened = serve.summarize(serve.run_stream(srv, open_shots, arr), open_shots, rate)
    srv.close()
    log(f"serving: capacity {closed['images_per_s']:.1f} img/s ({closed['Gterm_per_s']:.0f} Gterm/s); "
        f"at {load:.2f} load p50 {opened['p50_ms']:.1f} ms p99 {opened['p99_ms']:.1f} ms")
    # the same closed loop with the water-like background added to every image
    srv = xrt.Server(fh, hbm_budget=16 << 30, max_resident=64, precision="mixed",
                     background=synth.water_background())
    serve.run_stream(srv, cap_shots[:2], np.zeros(2))
    with_bg = serve.summarize(serve.run_stream(srv, cap_shots, np.zeros(n_cap)), cap_shots)
    srv.close()
    log(f"serving with the background: capacity {with_bg['images_per_s']:.1f} img/s")
    return {"workload": "served stream: log-uniform ROI, 1-100 sources, 1-200 domains, N in [5,40], mixed",
            "closed_loop": closed, "poisson": opened, "load": load, "closed_loop_with_background": with_bg}


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


def serving_sweep(n_cap=200, n_open=1000, loads=(0.5, 0.8, 0.95), small_budget=256 << 20):
    """The served stream at several offered loads: capacity from n_cap shots
    submitted at once, then n_open Poisson arrivals at each load x capacity;
    finally the capacity again under a small HBM budget, which admits fewer
    shots at once.  Several minutes of GPU time: not part of the default run."""
    import numpy as np
    import synth
    from paper_2205_07976_amd import serve, xrt
    base = synth.full_shot()
    fh = xrt.Fhkl.from_shot(base)
    rng = np.random.default_rng(14)

    def progress(tag, n):
        def cb(i, t, count=[0]):
            count[0] += 1
            if count[0] % 100 == 0 or count[0] == n:
                log(f"  {tag}: {count[0]}/{n} shots done")
        return cb

    out = {"workload": "served stream: log-uniform ROI, 1-100 sources, 1-200 domains, N in [5,40], mixed"}
    for name, budget in (("budget_16GiB", 16 << 30), (f"budget_{small_budget >> 20}MiB", small_budget)):
        srv = xrt.Server(fh, hbm_budget=budget, max_resident=64, precision="mixed")
        cap_shots = [synth.served_shot(rng, base.F, base.hkl_min) for _ in range(n_cap)]
        serve.run_stream(srv, cap_shots[:2], np.zeros(2))
        closed = serve.summarize(serve.run_stream(srv, cap_shots, np.zeros(n_cap),
                                                  on_done=progress(f"{name} capacity", n_cap)), cap_shots)
        log(f"{name}: capacity {closed['images_per_s']:.2f} img/s ({closed['Gterm_per_s']:.0f} Gterm/s)")
        res = {"closed_loop": closed}
        if name == "budget_16GiB":
            for load in loads:
                shots = [synth.served_shot(rng, base.F, base.hkl_min) for _ in range(n_open)]
                rate = load * closed["images_per_s"]
                arr = serve.poisson_arrivals(np.random.default_rng(int(load * 100)), n_open, rate)
                opened = serve.summarize(serve.run_stream(srv, shots, arr, on_done=progress(f"load {load}", n_open)),
                                         shots, rate)
                log(f"{name} at {load:.2f} load: p50 {opened['p50_ms']:.1f} ms p99 {opened['p99_ms']:.1f} ms, "
                    f"{opened['Gterm_per_s']:.0f} Gterm/s")
                res[f"poisson_{load:.2f}"] = opened
        srv.close()
        out[name] = res
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision form")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the regions-of-interest adjoint")
    ap.add_argument("--no-background", action="store_true", help="skip the background of an amorphous scatterer")
    ap.add_argument("--no-serve", action="store_true", help="skip the served shot stream")
    ap.add_argument("--serve-sweep", action="store_true",
                    help="also serve 1000 Poisson shots at 0.5, 0.8 and 0.95 x capacity and measure the "
                         "capacity under a 256 MiB budget (several minutes)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="finish with one device-to-device copy of this many MiB (a kernel of known "
                         "traffic that calibrates the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); shots would be sharded "
              "one per GPU with no exchange, which this build does not launch.", file=sys.stderr)
        return 2

    import torch
    import synth
    from paper_2205_07976_amd import xrt

    torch.cuda.set_device(0)
    shot = synth.full_shot()
    fh = xrt.Fhkl.from_shot(shot)
    terms = shot.n_terms
    log(f"full-size shot: {terms:.4e} terms; fp64 warmup {args.warmup} steps {args.steps}")

    img64, wall, ev = time_form(shot, fh, "fp64", args.steps, args.warmup)
    ms = 1e3 * wall / args.steps
    kern_ms = sum(ev) / len(ev)
    value = terms / (wall / args.steps) / 1e9
    ach = C_ALG["fp64"] * terms / (kern_ms * 1e-3)
    res = {
        "metric": "pixel-term evaluations/s (G/s) vs FP32 VALU peak; p50/p99 shot latency",
        "value": value, "unit": "Gterm/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "full-size shot, binary64: 2463x2527 px, oversample 2, 3 layers, "
                               "100 sources, 50 mosaic domains, sincg N=20, Fhkl [-60,60]^3",
                   "pixels": shot.n_pixels, "terms_per_pixel": shot.terms_per_pixel, "terms": terms},
        "roofline": {"bound": "alu", "achieved": ach / 1e12, "peak": PEAK_OPS / 1e12,
                     "unit": "T fp32-lane-op/s", "frac": ach / PEAK_OPS, "traffic": TRAFFIC_FP64,
                     "kernel": "spots_kernel<FP64,SINCG>", "kernel_ms": kern_ms,
                     "c_alg_per_term": C_ALG["fp64"]},
    }
    log(f"fp64: {ms:.1f} ms/step (events {kern_ms:.1f} ms), {value:.1f} Gterm/s, "
        f"roofline frac {ach / PEAK_OPS:.3f}")

    if not args.no_mixed:
        img32, wall32, ev32 = time_form(shot, fh, "mixed", args.steps, args.warmup)
        k32 = sum(ev32) / len(ev32)
        v32 = terms / (wall32 / args.steps) / 1e9
        a32 = C_ALG["mixed"] * terms / (k32 * 1e-3)
        emax, erms = mixed_error(shot, img32.cpu().numpy())
        res["mixed"] = {"value": v32, "unit": "Gterm/s", "ms_per_step": 1e3 * wall32 / args.steps,
                        "kernel_ms": k32, "frac": a32 / PEAK_OPS, "speedup_vs_fp64": v32 / value,
                        "max_rel_err": emax, "rms_rel_err": erms, "err_sample": "256 seeded pixels"}
        log(f"mixed: {1e3 * wall32 / args.steps:.1f} ms/step, {v32:.1f} Gterm/s, max rel err {emax:.2e}")

    # a small region of the same shot: its sums are split over many
    # workgroups (a 64 x 64 region is only 16 tiles)
    small = shot.replace(roi=(1200, 1264, 1250, 1314))
    res["small_roi"] = {"workload": "64x64 region of the full-size shot (2.46e8 terms, split sums)"}
    for prec in ("fp64", "mixed"):
        _, wall_s, ev_s = time_form(small, fh, prec, max(args.steps, 5), 1)
        ms_s = sum(ev_s) / len(ev_s)
        res["small_roi"][prec] = {"ms": ms_s, "Gterm_s": small.n_terms / ms_s / 1e6}
        log(f"small ROI {prec}: {ms_s:.2f} ms, {small.n_terms / ms_s / 1e6:.0f} Gterm/s")

    if not args.no_background:
        res["background"] = background_bench(shot, args.steps)
        res["background"]["image_fp64_ms"] = kern_ms + res["background"]["fp64"]["ms"]

    if not args.no_background:
        res["ensemble"] = ensemble_bench(shot, args.steps)

    if not args.no_adjoint:
        res["adjoint"] = adjoint_bench(args.steps)

    if not args.no_serve:
        res["serving"] = serving_bench()
        res["p50_shot_latency_ms"] = res["serving"]["poisson"]["p50_ms"]
        res["p99_shot_latency_ms"] = res["serving"]["poisson"]["p99_ms"]
        res["serving_io"] = serving_io_bench()
    if args.serve_sweep:
        res["serving_sweep"] = serving_sweep()

    if args.copy_mib:
        n = args.copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_mib} MiB read + {args.copy_mib} MiB written")

    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(shot)
        log(f"cpu oracle: {res['cpu_baseline']}")
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
