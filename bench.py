#!/usr/bin/env python3
"""Throughput of separable W-projection gridding + degridding on one MI355X.

Workload (the array-scale configuration): 4096^2 grid, 3 deg field, 64
antennas in an 8 km disc, dec -30 deg, 8 h earth-rotation track in 10 s dumps,
16 channels -> 92,897,280 visibilities; 128 w-planes over +/- max|w|,
support 15, oversample 8, PSWF taper, complex Gaussian V, unit weights; all
synthetic and seeded, resident in HBM before the timed region.

One step is the whole hot path over that batch, through the C ABI:
  1. table generation for the batch's w range       (sepw_kernels_set_wrange)
  2. quantise + w-plane + tile counting sort        (sepw_plan_rebin)
  3. gridding -> FFT -> grid correction (x n)        (sepw_grid, SEPW_MUL_N)
  4. model image correction (/ n) -> FFT -> degrid   (sepw_degrid, SEPW_DIV_N)
value = visibilities / step time (Mvis/s, gridded + degridded).

Per-stage times come from HIP events the library records on its launch stream
(sepw_timing_*); the roofline entry is for the dominant kernel.  The other
forms (FP16 / BF16 operands, the batched facet launch, the W-stacking hybrid,
the 2D correction table, channel-shared coordinates, W snapshots, the
differentiable prediction) are reported beside the FP32 line, each with its
error against the oracle.  The CPU baseline times the FP64 NumPy oracle on a
bounded sample of the same workload.
"""
import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Mvis/s gridded+degridded (FP32 vs FP16-MFMA at stated RMS err); % roofline"
PEAK_FP32_MFMA_TFLOPS = 157.3      # MI355X dense FP32 matrix peak
PEAK_HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_grid_degrid_array4096_fp32.md")


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` ("grid" or "degrid") from the committed
    FETCH_SIZE / WRITE_SIZE counter summary (calibrated against a kernel of known
    traffic), or None when the kernel's sources have changed since the counters
    were taken or no summary is present."""
    import hashlib
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    if not m:
        return None
    entry = json.loads(m.group(1))["kernels"].get(kernel)
    if entry is None:
        return None
    h = hashlib.sha256()
    for f in entry["sources"]:
        try:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        except OSError:
            return None
    return entry["bytes_per_launch"] if h.hexdigest() == entry["sources_sha256"] else None


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_worker(args):
    """One worker of the CPU baseline: quantise, grid (private FP64 grid) and
    degrid (from the shared pre-corrected grid) one chunk of visibilities."""
    import numpy as np
    from multiprocessing import shared_memory
    from threadpoolctl import threadpool_limits

    import oracle
    u, v, w, y, T, g = args
    with threadpool_limits(limits=1):
        N, fov, S, O, P, w_lo, w_hi, shm_name = g
        shm = shared_memory.SharedMemory(name=shm_name)
        try:
            Gh = np.ndarray((N, N), np.complex128, buffer=shm.buf)
            q = oracle.quantise.quantise(u, v, w, N, fov, O, S, P, w_lo, w_hi, 17 - S)
            G = oracle.gridder.grid_separable(q, y, T, N, S)
            Vp = oracle.gridder.degrid_separable(q, Gh, T, N, S)
            del Gh
        finally:
            shm.close()
    return G, len(Vp)


def cpu_baseline(d, n_sample, workers):
    """Oracle (FP64 NumPy) on the first n_sample visibilities, over a pool of
    worker processes: tables and both FFT corrections in the parent, the
    visibilities in equal chunks, each worker quantising, gridding into a
    private grid and degridding its chunk; the grids summed at the end."""
    import multiprocessing as mp
    from multiprocessing import shared_memory

    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle
    N, fov, S, O, P = d["N"], d["fov"], d["S"], d["O"], d["P"]
    sl = slice(0, n_sample)
    u, v, w = d["u"][sl], d["v"][sl], d["w"][sl]
    y = d["V"][sl].astype(np.complex128) * d["W"][sl]
    rng = np.random.default_rng(7)
    X = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    ctx = mp.get_context("spawn")   # fresh interpreters: the parent holds the GPU
    shm = shared_memory.SharedMemory(create=True, size=N * N * 16)
    try:
        with ctx.Pool(workers) as pool:
            pool.map(abs, range(workers))           # workers started before the clock
            with threadpool_limits(limits=1):
                t0 = time.perf_counter()
                c1 = oracle.pswf.taper_c1(N, fov, S)
                T = oracle.tables.separable_table(
                    oracle.tables.w_plane_centres(P, d["w_lo"], d["w_hi"]), N, fov, S, O, c1)
                Gh = np.ndarray((N, N), np.complex128, buffer=shm.buf)
                Gh[...] = oracle.imaging.grid_from_image(X, c1, fov, n_power=-1)
                del Gh
                g = (N, fov, S, O, P, d["w_lo"], d["w_hi"], shm.name)
                bounds = np.linspace(0, n_sample, workers + 1).astype(np.int64)
                jobs = [(u[a:b], v[a:b], w[a:b], y[a:b], T, g)
                        for a, b in zip(bounds[:-1], bounds[1:])]
                G = None
                for Gw, _ in pool.imap_unordered(_oracle_worker, jobs):
                    G = Gw if G is None else G + Gw
                img = oracle.imaging.image_from_grid(G, c1, fov, n_power=1)
                t1 = time.perf_counter()
    finally:
        shm.close()
        shm.unlink()
    del img
    secs = t1 - t0
    return {"value": round(n_sample / secs / 1e6, 4), "unit": "Mvis/s", "cores": workers,
            "kind": "oracle", "cpu": _cpu_model(), "cpu_count": os.cpu_count(),
            "sample": "first %d visibilities of the workload (of %d); tables + F-/correction, then "
                      "quantise + grid + degrid in %d worker processes (private FP64 grids, "
                      "summed), F+/correction; FP64 NumPy, %.1f s"
                      % (n_sample, len(d["u"]), workers, secs),
            "seconds": round(secs, 2)}


def accuracy_64(_lib, torch):
    """Relative RMS error of each precision against the FP64 oracle on the
    64^2, 2,000-visibility workload: dirty image over the inner half and
    visibilities predicted from an inner-half model."""
    import numpy as np

    import oracle
    from paper_1511_07152_amd import synth
    d = synth.accuracy_64()
    N, fov, S, O, P = d["N"], d["fov"], d["S"], d["O"], d["P"]
    c1 = oracle.pswf.taper_c1(N, fov, S)
    T = oracle.tables.separable_table(oracle.tables.w_plane_centres(P, d["w_lo"], d["w_hi"]),
                                      N, fov, S, O, c1)
    rng = np.random.default_rng(64)
    X = np.zeros((N, N), complex)
    X[N // 4:3 * N // 4, N // 4:3 * N // 4] = (rng.standard_normal((N // 2, N // 2))
                                               + 1j * rng.standard_normal((N // 2, N // 2)))
    dev = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dt)  # noqa: E731
    inner = slice(N // 4, 3 * N // 4)
    out = {}
    for prec in ("fp32", "fp16", "bf16"):
        K = _lib.Kernels(N, fov, S, O, P, d["w_lo"], d["w_hi"], precision=prec)
        plan = _lib.Plan(K, dev(d["u"], torch.float64), dev(d["v"], torch.float64),
                         dev(d["w"], torch.float64))
        img = _lib.grid(plan, dev(d["V"], torch.complex64), dev(d["W"], torch.float32),
                        flags=_lib.MUL_N).cpu().numpy()
        Vp = _lib.degrid(plan, dev(X, torch.complex64), flags=_lib.DIV_N).cpu().numpy()
        q = oracle.quantise.quantise(d["u"], d["v"], d["w"], N, fov, O, S, P, d["w_lo"], d["w_hi"],
                                     plan.tile_size)
        ref_img = oracle.imaging.image_from_grid(
            oracle.gridder.grid_separable(q, d["V"] * d["W"], T, N, S), c1, fov, n_power=1)
        ref_v = oracle.gridder.degrid_separable(q, oracle.imaging.grid_from_image(X, c1, fov, -1),
                                                T, N, S)
        e_img = np.linalg.norm((img - ref_img)[inner, inner]) / np.linalg.norm(ref_img[inner, inner])
        e_vis = np.linalg.norm(Vp - ref_v) / np.linalg.norm(ref_v)
        out[prec] = {"image": float("%.3g" % e_img), "vis": float("%.3g" % e_vis)}
    return out


def wstack_form(_lib, torch, d, u, v, w, V, W, model, steps):
    """W-stacking hybrid (Section 4.3) on the array-scale workload: 16 uniform
    w-slices over the same w range, 8 residual planes per slice (the plain
    path's plane density), grid (x n) + degrid (/ n) per step; plus its parity
    with the oracle on the 64^2 accuracy workload (4 slices, 2 residual planes)."""
    import numpy as np

    import oracle
    from paper_1511_07152_amd import synth
    N, fov, S, O = d["N"], d["fov"], d["S"], d["O"]
    ns, P = 16, 8
    h = (d["w_hi"] - d["w_lo"]) / (2 * ns)
    K = _lib.Kernels(N, fov, S, O, P, -h, h)
    t = time.perf_counter()
    ws = _lib.WStack(K, ns, d["w_lo"], d["w_hi"], u, v, w)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t
    img = torch.empty((N, N), dtype=torch.complex64, device="cuda")
    vis_out = torch.empty(ws.nvis, dtype=torch.complex64, device="cuda")

    def step():
        ws.grid(V, W, flags=_lib.MUL_N, out=img)
        ws.degrid(model, flags=_lib.DIV_N, out=vis_out)

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    res = {"workload": "array-scale, %d w-slices x %d residual planes, S=%d, O=%d" % (ns, P, S, O),
           "slices": ns, "residual_planes": P, "ms_per_step": round(ms, 3),
           "Mvis_per_s": round(ws.nvis / (ms * 1e-3) / 1e6, 2), "create_s": round(t_create, 3)}
    ws.close()
    K.close()
    # parity with the oracle at 64^2
    a = synth.accuracy_64()
    N2, fov2, S2, O2 = a["N"], a["fov"], a["S"], a["O"]
    ns2, P2 = 4, 2
    h2 = (a["w_hi"] - a["w_lo"]) / (2 * ns2)
    dev = lambda x, dt: torch.as_tensor(np.ascontiguousarray(x)).to("cuda", dt)  # noqa: E731
    K2 = _lib.Kernels(N2, fov2, S2, O2, P2, -h2, h2)
    ws2 = _lib.WStack(K2, ns2, a["w_lo"], a["w_hi"], dev(a["u"], torch.float64),
                      dev(a["v"], torch.float64), dev(a["w"], torch.float64))
    got = ws2.grid(dev(a["V"], torch.complex64), dev(a["W"], torch.float32),
                   flags=_lib.MUL_N).cpu().numpy()
    c1 = oracle.pswf.taper_c1(N2, fov2, S2)
    want = oracle.wstack.image(a["u"], a["v"], a["w"], a["V"] * a["W"], N2, fov2, S2, O2, P2, ns2,
                               a["w_lo"], a["w_hi"], c1, n_power=1)
    q = slice(N2 // 4, 3 * N2 // 4)
    res["rel_rms_err_image_64"] = float("%.3g" % (np.linalg.norm((got - want)[q, q])
                                                  / np.linalg.norm(want[q, q])))
    ws2.close()
    K2.close()
    return res


def correction_form(_lib, torch, d, u, v, w, V, W, model, steps, Sc=13, Oc=8):
    """The correction table F_w - F~_w (Section 6) attached to the array-scale
    kernels (S_c = 13, O_c = 8): its FP64 generation for the 128 planes, then
    grid (x n) + degrid (/ n) per step with the correction passes; plus, on a
    wide-field 64^2 case (fov 0.4, |w| <= 20, S = 15, 300 visibilities), the
    GPU image's error against the exact DFT with and without the correction and
    its parity with the oracle."""
    import numpy as np

    import oracle
    N, fov, S, O, P = d["N"], d["fov"], d["S"], d["O"], d["P"]
    K = _lib.Kernels(N, fov, S, O, P, d["w_lo"], d["w_hi"])
    torch.cuda.synchronize()
    t = time.perf_counter()
    K.set_correction(Sc, Oc)
    torch.cuda.synchronize()
    table_ms = (time.perf_counter() - t) * 1e3
    plan = _lib.Plan(K, u, v, w)
    img = torch.empty((N, N), dtype=torch.complex64, device="cuda")
    vis_out = torch.empty(plan.nvis, dtype=torch.complex64, device="cuda")

    def step():
        _lib.grid(plan, V, W, flags=_lib.MUL_N, out=img)
        _lib.degrid(plan, model, flags=_lib.DIV_N, out=vis_out)

    step()
    torch.cuda.synchronize()
    _lib.timing_enable(True)
    _lib.timing_collect()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    _lib.timing_enable(False)
    st = _lib.timing_collect()
    res = {"workload": "array-scale, correction S_c=%d O_c=%d beside S=%d O=%d, %d planes"
                       % (Sc, Oc, S, O, P),
           "table_generation_ms": round(table_ms, 2), "ms_per_step": round(ms, 3),
           "Mvis_per_s": round(plan.nvis / (ms * 1e-3) / 1e6, 2),
           "stages_ms_per_step": {k: round(v_ / steps, 4) for k, (v_, n) in st.items() if n}}
    plan.close()
    K.close()
    # wide field at 64^2: error against the exact DFT, and oracle parity
    n2, fov2, S2, O2, P2, wmax = 64, 0.4, 15, 8, 4, 20.0
    rng = np.random.default_rng(3)
    cells = n2 / 2 - S2
    u2 = rng.uniform(-cells, cells, 300) / fov2
    v2 = rng.uniform(-cells, cells, 300) / fov2
    w2 = rng.uniform(-wmax, wmax, 300)
    y2 = rng.standard_normal(300) + 1j * rng.standard_normal(300)
    dev = lambda x, dt: torch.as_tensor(np.ascontiguousarray(x)).to("cuda", dt)  # noqa: E731
    K2 = _lib.Kernels(n2, fov2, S2, O2, P2, -wmax, wmax)
    p2 = _lib.Plan(K2, dev(u2, torch.float64), dev(v2, torch.float64), dev(w2, torch.float64))
    sep = _lib.grid(p2, dev(y2, torch.complex64)).cpu().numpy()
    K2.set_correction(Sc, Oc)
    cor = _lib.grid(p2, dev(y2, torch.complex64)).cpu().numpy()
    c1 = oracle.pswf.taper_c1(n2, fov2, S2)
    q = oracle.quantise.quantise(u2, v2, w2, n2, fov2, O2, S2, P2, -wmax, wmax, p2.tile_size)
    wc = oracle.tables.w_plane_centres(P2, -wmax, wmax)
    keep = ~q["dropped"]
    uh, vh = oracle.quantise.dequantised(q, n2, fov2, O2)
    ref = oracle.dft.dirty(uh[keep], vh[keep], wc[q["k"][keep]], y2[keep], n2, fov2,
                           oracle.dft.phase_screen(n2, fov2, "exact"))
    T = oracle.tables.separable_table(wc, n2, fov2, S2, O2, c1)
    C = oracle.correction.correction_table(wc, n2, fov2, Sc, Oc, c1)
    want = oracle.imaging.image_from_grid(oracle.correction.grid(q, y2, T, C, n2, S2, O2, Sc, Oc),
                                          c1, fov2)
    i = slice(n2 // 4, 3 * n2 // 4)
    err = lambda a, b: float("%.3g" % (np.linalg.norm((a - b)[i, i]) / np.linalg.norm(b[i, i])))  # noqa: E731
    res["wide_field_64"] = {"err_vs_exact_dft_separable": err(sep, ref),
                            "err_vs_exact_dft_corrected": err(cor, ref),
                            "rel_rms_err_vs_oracle": err(cor, want)}
    p2.close()
    K2.close()
    return res


def channel_form(_lib, torch, d, u, v, w, V, W, model, steps):
    """Channel-shared coordinates on the array-scale workload: the same step as
    the FP32 line (tables, rebin, grid x n, degrid / n) with the plan rebinned
    from uvw per (baseline, time) row in metres and the 16 channel
    frequencies (24 / 16 B of coordinates per visibility instead of 24), and
    the difference of its image from the per-visibility plan's."""
    import numpy as np
    N, fov, S, O, P = d["N"], d["fov"], d["S"], d["O"], d["P"]
    uvw = torch.as_tensor(np.ascontiguousarray(d["uvw_m"])).to("cuda", torch.float64)
    freq = torch.as_tensor(np.ascontiguousarray(d["freqs"])).to("cuda", torch.float64)
    K = _lib.Kernels(N, fov, S, O, P, d["w_lo"], d["w_hi"])
    plan = _lib.Plan.from_channels(K, uvw, freq)
    img = torch.empty((N, N), dtype=torch.complex64, device="cuda")
    vis_out = torch.empty(plan.nvis, dtype=torch.complex64, device="cuda")

    def step():
        K.set_wrange(d["w_lo"], d["w_hi"])
        plan.rebin_channels(uvw, freq)
        _lib.grid(plan, V, W, flags=_lib.MUL_N, out=img)
        _lib.degrid(plan, model, flags=_lib.DIV_N, out=vis_out)

    step()
    torch.cuda.synchronize()
    _lib.timing_enable(True)
    _lib.timing_collect()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    _lib.timing_enable(False)
    st = _lib.timing_collect()
    ref_plan = _lib.Plan(K, u, v, w)
    ref = _lib.grid(ref_plan, V, W, flags=_lib.MUL_N)
    diff = float((torch.linalg.norm(img - ref) / torch.linalg.norm(ref)).item())
    res = {"workload": "array-scale, uvw per row (%d rows x %d channels)"
                       % (uvw.shape[0], freq.numel()),
           "ms_per_step": round(ms, 3), "Mvis_per_s": round(plan.nvis / (ms * 1e-3) / 1e6, 2),
           "quantise_ms": round(st["quantise"][0] / steps, 4),
           "image_rel_diff_vs_per_visibility_plan": float("%.3g" % diff),
           "dropped": plan.n_dropped, "dropped_per_visibility_plan": ref_plan.n_dropped}
    ref_plan.close()
    plan.close()
    K.close()
    return res


def wsnap_form(_lib, torch, d, u, v, w, V, W, model, steps, n_snap=16, planes=16):
    """W snapshots (Section 4.2) on the array-scale workload: 16 snapshots of
    30 min (contiguous in the time-ordered data), a plane fitted per snapshot,
    16 residual planes, grid (x n) + degrid (/ n) per step; plus parity with
    the oracle on a 64^2 case whose five snapshots tilt by up to 2.5."""
    import numpy as np

    import oracle
    N, fov, S, O = d["N"], d["fov"], d["S"], d["O"]
    nvis = len(d["u"])
    offs = [nvis * i // n_snap for i in range(n_snap + 1)]
    K = _lib.Kernels(N, fov, S, O, planes, -1.0, 1.0)
    t = time.perf_counter()
    ws = _lib.WSnap(K, offs, u, v, w)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t
    img = torch.empty((N, N), dtype=torch.complex64, device="cuda")
    vis_out = torch.empty(nvis, dtype=torch.complex64, device="cuda")

    def step():
        ws.grid(V, W, flags=_lib.MUL_N, out=img)
        ws.degrid(model, flags=_lib.DIV_N, out=vis_out)

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    h = ws.plane(0)[1]
    res = {"workload": "array-scale, %d snapshots x %d residual planes, S=%d, O=%d" % (n_snap, planes, S, O),
           "ms_per_step": round(ms, 3), "Mvis_per_s": round(nvis / (ms * 1e-3) / 1e6, 2),
           "create_s": round(t_create, 3), "residual_w_max": round(h, 2),
           "full_w_max": round(float(d["w_hi"]), 2), "dropped": ws.n_dropped}
    ws.close()
    K.close()
    # parity with the oracle at 64^2
    rng = np.random.default_rng(64_000)
    n2, fov2, S2, O2, P2, sizes = 64, 0.4, 7, 8, 4, (700, 0, 1, 900, 500)
    cells = n2 / 2 - 6
    parts = []
    for n in sizes:
        dd = rng.uniform(-2.5, 2.5, 2)
        a = rng.uniform(-cells, cells, (2, n)) / fov2
        parts.append((a[0], a[1], dd[0] * a[0] + dd[1] * a[1] + rng.normal(0, 2.0, n)))
    u2, v2, w2 = (np.concatenate([p_[k] for p_ in parts]) for k in range(3))
    y2 = rng.standard_normal(len(u2)) + 1j * rng.standard_normal(len(u2))
    offs2 = [0] + list(np.cumsum(sizes))
    dev = lambda x, dt: torch.as_tensor(np.ascontiguousarray(x)).to("cuda", dt)  # noqa: E731
    K2 = _lib.Kernels(n2, fov2, S2, O2, P2, -1.0, 1.0)
    ws2 = _lib.WSnap(K2, offs2, dev(u2, torch.float64), dev(v2, torch.float64), dev(w2, torch.float64))
    got = ws2.grid(dev(y2, torch.complex64), flags=_lib.MUL_N).cpu().numpy()
    c1 = oracle.pswf.taper_c1(n2, fov2, S2)
    want = oracle.wsnap.image(u2, v2, w2, y2, offs2, n2, fov2, S2, O2, P2, c1, n_power=1)
    q = slice(n2 // 4, 3 * n2 // 4)
    res["rel_rms_err_image_64"] = float("%.3g" % (np.linalg.norm((got - want)[q, q])
                                                  / np.linalg.norm(want[q, q])))
    ws2.close()
    K2.close()
    return res


def differentiation_form(_lib, torch, steps):
    """The differentiation workload: a 2048^2 real model, 4,285,440 visibilities
    (32 antennas, 4 km, 6 h in 20 s dumps, 8 channels), 64 planes, S = 15:
    V_t = A x_true + complex noise of 0.1 rms(A x_true); one step is
    chi^2(Predict(x)) and its gradient (degrid forward, gridding adjoint
    backward) at x = 0.9 x_true; plus the gradient's parity with the oracle's
    on a 64^2 case."""
    import numpy as np

    import oracle
    from paper_1511_07152_amd import autograd, synth
    d = synth.model_2048()
    N, fov, S, O, P = d["N"], d["fov"], d["S"], d["O"], d["P"]
    dev = lambda x, dt: torch.as_tensor(np.ascontiguousarray(x)).to("cuda", dt)  # noqa: E731
    K = _lib.Kernels(N, fov, S, O, P, d["w_lo"], d["w_hi"])
    plan = _lib.Plan(K, dev(d["u"], torch.float64), dev(d["v"], torch.float64),
                     dev(d["w"], torch.float64))
    xt = dev(d["x"], torch.float32)
    with torch.no_grad():
        v0 = autograd.predict(xt, plan)
        sigma = float(torch.sqrt(torch.mean(torch.abs(v0) ** 2)).item()) * 0.1
        Vt = v0 + sigma * dev(d["noise"], torch.complex64) / np.sqrt(2.0)
    W = dev(d["W"], torch.float32)

    def step():
        x = (0.9 * xt).requires_grad_(True)
        loss = autograd.chi2(autograd.predict(x, plan), Vt, W)
        loss.backward()
        return x.grad

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    res = {"workload": "2048^2 model, %d visibilities, %d planes, S=%d, O=%d" % (plan.nvis, P, S, O),
           "ms_per_step": round(ms, 3), "Mvis_per_s": round(plan.nvis / (ms * 1e-3) / 1e6, 2)}
    plan.close()
    K.close()
    # gradient parity at 64^2
    rng = np.random.default_rng(64_001)
    n2, fov2, S2, O2, P2, nv = 64, float(np.radians(2.0)), 7, 8, 8, 3000
    u2, v2 = rng.uniform(-26, 26, (2, nv)) / fov2
    w2 = rng.uniform(-200, 200, nv)
    x2 = np.zeros((n2, n2))
    x2[n2 // 4:3 * n2 // 4, n2 // 4:3 * n2 // 4] = rng.standard_normal((n2 // 2, n2 // 2))
    Vt2 = rng.standard_normal(nv) + 1j * rng.standard_normal(nv)
    W2 = rng.uniform(0.5, 2.0, nv)
    K2 = _lib.Kernels(n2, fov2, S2, O2, P2, -200.0, 200.0)
    p2 = _lib.Plan(K2, dev(u2, torch.float64), dev(v2, torch.float64), dev(w2, torch.float64))
    x = dev(x2, torch.float32).requires_grad_(True)
    autograd.chi2(autograd.predict(x, p2), dev(Vt2, torch.complex64), dev(W2, torch.float32)).backward()
    c1 = oracle.pswf.taper_c1(n2, fov2, S2)
    q = oracle.quantise.quantise(u2, v2, w2, n2, fov2, O2, S2, P2, -200.0, 200.0, p2.tile_size)
    T = oracle.tables.separable_table(oracle.tables.w_plane_centres(P2, -200.0, 200.0), n2, fov2,
                                      S2, O2, c1)
    want = oracle.chi2.chi2_grad(oracle.chi2.SeparableOperator(q, T, c1, n2, S2, fov2), x2, Vt2, W2)
    got = x.grad.cpu().numpy()
    i = slice(n2 // 4, 3 * n2 // 4)
    res["rel_rms_err_gradient_64"] = float("%.3g" % (np.linalg.norm((got - want)[i, i])
                                                     / np.linalg.norm(want[i, i])))
    p2.close()
    K2.close()
    return res


def batching_form(_lib, torch, args):
    """36 image-plane facets (6 x 6 over 10 deg, 1024^2 each, S = 11, 64 planes,
    log-normal visibility counts): one persistent sepw_grid_batched launch (its
    work-item length and launch width picked first by sepw_autotune_batched)
    vs one sepw_grid launch per facet, both through FFT and correction."""
    import numpy as np

    from paper_1511_07152_amd import synth
    d = synth.facets_36()
    N, fov, S, O, P = d["N"], d["fov"], d["S"], d["O"], d["P"]
    dev = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dt)  # noqa: E731
    Ks, plans, vis, wts, outs = [], [], [], [], []
    nvis = 0
    for jb in d["jobs"]:
        wmax = float(np.max(np.abs(jb["w"]))) * (1 + 1e-9) + 1e-9
        K = _lib.Kernels(N, fov, S, O, P, -wmax, wmax, facet=(jb["l0"], jb["m0"]))
        Ks.append(K)
        plans.append(_lib.Plan(K, dev(jb["u"], torch.float64), dev(jb["v"], torch.float64),
                               dev(jb["w"], torch.float64)))
        vis.append(dev(jb["V"], torch.complex64))
        wts.append(dev(jb["W"], torch.float32))
        outs.append(torch.empty((N, N), dtype=torch.complex64, device="cuda"))
        nvis += len(jb["u"])
    dropped = sum(p.n_dropped for p in plans)

    def batched():
        _lib.grid_batched(plans, vis, wts, flags=_lib.MUL_N, outs=outs)

    def per_job():
        for p, x, wt, o in zip(plans, vis, wts, outs):
            _lib.grid(p, x, wt, flags=_lib.MUL_N, out=o)

    def item_slots(n):
        for p in plans:
            p.set_item_slots(n)

    t0 = time.perf_counter()
    slots, width = _lib.autotune_batched(plans, vis, wts, outs=outs)
    tune_s = time.perf_counter() - t0
    res = {"workload": "36 facets 6x6 over 10 deg, 1024^2, S=11, O=8, 64 planes",
           "nvis": nvis, "dropped": dropped,
           "autotuned": {"item_slots": slots, "blocks_per_cu": width, "seconds": round(tune_s, 2)}}
    for name, fn in (("batched", batched), ("per_facet", per_job)):
        if name == "per_facet":
            item_slots(1024)   # per-facet launches with the default work-item length
        for _ in range(max(args.warmup, 1)):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        res[name] = {"ms": round(ms, 3), "Mvis_per_s": round(nvis / (ms * 1e-3) / 1e6, 2)}
    log("batched facets: %s" % res)
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--dump-s", type=float, default=10.0, help="dump time (10 s: 92.9M vis)")
    ap.add_argument("--cpu-sample", type=int, default=12_000_000)
    ap.add_argument("--cpu-workers", type=int, default=min(16, os.cpu_count() or 1),
                    help="worker processes of the CPU baseline (at most the host's CPU share)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fp32-only", action="store_true",
                    help="skip the FP16/BF16 MFMA forms and their accuracy check")
    ap.add_argument("--no-weights", action="store_true",
                    help="pass W = NULL (unit weights implied) instead of an array of ones")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1511_07152_amd import _lib, synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    _lib.load()

    t = time.perf_counter()
    d = synth.array_4096(dump_s=args.dump_s)
    nvis = len(d["u"])
    log("generated %d visibilities in %.1f s" % (nvis, time.perf_counter() - t))
    N, fov, S, O, P = d["N"], d["fov"], d["S"], d["O"], d["P"]

    dev = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dt)  # noqa: E731
    u, v, w = dev(d["u"], torch.float64), dev(d["v"], torch.float64), dev(d["w"], torch.float64)
    V, W = dev(d["V"], torch.complex64), dev(d["W"], torch.float32)
    g = torch.Generator(device="cuda").manual_seed(1511)
    model = torch.randn((N, N), dtype=torch.complex64, device="cuda", generator=g)
    img = torch.empty((N, N), dtype=torch.complex64, device="cuda")
    vis_out = torch.empty(nvis, dtype=torch.complex64, device="cuda")

    def measure(precision):
        """Warm up, then time args.steps steps; returns (ms/step, stages, kept)."""
        K = _lib.Kernels(N, fov, S, O, P, d["w_lo"], d["w_hi"], precision=precision)
        plan = _lib.Plan(K, u, v, w)
        log("%s plan: %d kept, %d dropped, tile %d" % (precision, nvis - plan.n_dropped,
                                                       plan.n_dropped, plan.tile_size))

        def step():
            K.set_wrange(d["w_lo"], d["w_hi"])
            plan.rebin(u, v, w)
            _lib.grid(plan, V, None if args.no_weights else W, flags=_lib.MUL_N, out=img)
            _lib.degrid(plan, model, flags=_lib.DIV_N, out=vis_out)

        for i in range(args.warmup):
            step()
            torch.cuda.synchronize()
            log("%s warmup step %d done" % (precision, i))
        _lib.timing_enable(True)
        _lib.timing_collect()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _lib.timing_enable(False)
        stages = _lib.timing_collect()
        log("%s: timed %d steps in %.3f s" % (precision, args.steps, t1 - t0))
        kept = nvis - plan.n_dropped
        plan.close()
        K.close()
        return (t1 - t0) * 1e3 / args.steps, stages, kept

    ms_per_step, stages, kept = measure("fp32")
    value = nvis / (ms_per_step * 1e-3) / 1e6

    per_launch = {k: (ms / n if n else 0.0) for k, (ms, n) in stages.items()}
    flops = {"grid": kept * (8 * S * S + 6 * S + 2), "degrid": kept * (8 * S * S + 8 * S)}
    dom = max(("grid", "degrid"), key=lambda k: per_launch[k])
    achieved = flops[dom] / (per_launch[dom] * 1e-3) / 1e12
    roofline = {"kernel": dom, "bound": "mfma", "achieved": round(achieved, 2),
                "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_MFMA_TFLOPS, 4), "traffic": measured_traffic(dom),
                "traffic_unit": "bytes/launch",
                "avg_ms": round(per_launch[dom], 4)}

    forms = {}
    if not args.fp32_only:
        acc = accuracy_64(_lib, torch)
        forms["fp32"] = {"rel_rms_err": acc["fp32"]}
        for prec in ("fp16", "bf16"):
            ms, st, _ = measure(prec)
            forms[prec] = {"value": round(nvis / (ms * 1e-3) / 1e6, 2), "ms_per_step": round(ms, 3),
                           "grid_ms": round(st["grid"][0] / max(st["grid"][1], 1), 4),
                           "degrid_ms": round(st["degrid"][0] / max(st["degrid"][1], 1), 4),
                           "rel_rms_err": acc[prec]}

    if not args.fp32_only:
        forms["batched_facets"] = batching_form(_lib, torch, args)
        forms["w_stacking"] = wstack_form(_lib, torch, d, u, v, w, V, W, model, min(args.steps, 5))
        log("w-stacking: %s" % forms["w_stacking"])
        forms["correction_table"] = correction_form(_lib, torch, d, u, v, w, V, W, model,
                                                    min(args.steps, 5))
        log("correction table: %s" % forms["correction_table"])
        forms["channel_shared"] = channel_form(_lib, torch, d, u, v, w, V, W, model, args.steps)
        log("channel-shared coordinates: %s" % forms["channel_shared"])
        forms["w_snapshots"] = wsnap_form(_lib, torch, d, u, v, w, V, W, model, min(args.steps, 5))
        log("w-snapshots: %s" % forms["w_snapshots"])
        forms["differentiation"] = differentiation_form(_lib, torch, args.steps)
        log("differentiation: %s" % forms["differentiation"])

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "Mvis/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": "array-scale separable W-projection: 4096^2 grid, 3 deg, 64 antennas "
                               "8 km, 8 h, %g s dumps, 16 ch, 128 w-planes, S=15, O=8" % args.dump_s,
                   "nvis": nvis, "kept": kept, "grid": N, "support": S, "oversample": O,
                   "w_planes": P, "precision": "fp32"},
        "roofline": roofline,
        "stages_ms_per_step": {k: round(ms / args.steps, 4) for k, (ms, n) in stages.items()},
        # context: visibilities over the gridding + degridding kernel time alone
        # (binning, tables, FFT and correction left out)
        "grid_degrid_kernels_Mvis_per_s": round(
            nvis / ((per_launch["grid"] + per_launch["degrid"]) * 1e-3) / 1e6, 2),
    }
    if forms:
        out["precision_forms"] = forms
    if not args.no_cpu_baseline:
        del u, v, w
        t = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(d, min(args.cpu_sample, nvis), args.cpu_workers)
        log("cpu baseline in %.1f s" % (time.perf_counter() - t))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
