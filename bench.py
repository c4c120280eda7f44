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
differentiable prediction) are reported beside the FP32 line; the 16-bit
forms and the hybrids with the relative RMS difference of their outputs from
the FP32 step's on the same data (parity with the FP64 oracle is checked by
the tests).  Only the CPU baseline runs the oracle: it times the FP64 NumPy
oracle on a bounded sample of the same workload.
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


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_grid_degrid_array4096.md")


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


def rel_diff(torch, got, ref, inner=False):
    """Relative RMS difference ||got - ref|| / ||ref|| on the device in FP64
    (over the inner half of an image when inner is set), three significant
    digits."""
    if inner:
        n = ref.shape[0]
        q = slice(n // 4, 3 * n // 4)
        got, ref = got[q, q], ref[q, q]
    got, ref = got.to(torch.complex128), ref.to(torch.complex128)
    return float("%.3g" % (torch.linalg.norm(got - ref) / torch.linalg.norm(ref)).item())


class ExactDFT:
    """Exact references for sampled outputs of the array-scale step, in FP64
    with plain torch operations on the GPU (measurement only):
      * the dirty image of Section 2's equation with the exact w term, times n
        (the library's SEPW_MUL_N image), at npix pixels of the inner half:
        D(l, m) = n sum_i W_i V_i exp(2 pi i (u_i l + v_i m + w_i (n - 1)));
      * the prediction of an image X at nv visibilities (SEPW_DIV_N):
        V_i = sum_pixels X(l, m) / n exp(-2 pi i (u_i l + v_i m + w_i (n - 1))),
        X nonzero on the inner half only;
    with n - 1 = -(l^2 + m^2) / (1 + n).  Against these, an output's error
    holds every approximation of the method at once (the separable screen,
    the w-plane, the truncated support, the uv rounding to 1/O cell)."""

    def __init__(self, torch, d, u, v, w, V, W, X, npix=64, nv=256, seed=1511):
        import numpy as np
        N, fov = d["N"], d["fov"]
        dev = u.device
        rng = np.random.default_rng(seed)
        self.pq = rng.integers(N // 4, 3 * N // 4, (2, npix))
        self.vi = torch.as_tensor(rng.choice(u.numel(), nv, replace=False), device=dev)
        f64 = torch.float64
        lp = (torch.as_tensor(self.pq[0], device=dev, dtype=f64) - N / 2) * (fov / N)
        mq = (torch.as_tensor(self.pq[1], device=dev, dtype=f64) - N / 2) * (fov / N)
        r2 = lp * lp + mq * mq
        n = torch.sqrt(1.0 - r2)
        nm1 = -r2 / (1.0 + n)
        y = V.to(torch.complex128) * W.to(f64)
        D = torch.zeros(npix, dtype=torch.complex128, device=dev)
        step = 1 << 21
        for a in range(0, u.numel(), step):
            b = min(a + step, u.numel())
            ph = 2 * np.pi * (u[a:b, None] * lp + v[a:b, None] * mq + w[a:b, None] * nm1)
            D += (y[a:b, None] * torch.polar(torch.ones_like(ph), ph)).sum(0)
        self.image = D * n
        # prediction of X at the sampled visibilities, over the inner half
        q0, q1 = N // 4, 3 * N // 4
        li = (torch.arange(q0, q1, device=dev, dtype=f64) - N / 2) * (fov / N)
        L = li[None, :].expand(q1 - q0, -1).reshape(-1)
        M = li[:, None].expand(-1, q1 - q0).reshape(-1)
        r2 = L * L + M * M
        n = torch.sqrt(1.0 - r2)
        x = X[q0:q1, q0:q1].reshape(-1).to(torch.complex128) / n
        nm1 = -r2 / (1.0 + n)
        us, vs, ws = u[self.vi], v[self.vi], w[self.vi]
        P = torch.zeros(nv, dtype=torch.complex128, device=dev)
        step = 1 << 18
        for a in range(0, L.numel(), step):
            b = min(a + step, L.numel())
            ph = -2 * np.pi * (us[:, None] * L[a:b] + vs[:, None] * M[a:b] + ws[:, None] * nm1[a:b])
            P += (x[a:b] * torch.polar(torch.ones_like(ph), ph)).sum(1)
        self.vis = P

    def errors(self, torch, img, vis):
        """Relative RMS error of an image (sampled pixels) and predictions
        (sampled visibilities) against the exact references."""
        got = img[self.pq[1], self.pq[0]].to(torch.complex128)
        gv = vis[self.vi].to(torch.complex128)
        e_i = torch.linalg.norm(got - self.image) / torch.linalg.norm(self.image)
        e_v = torch.linalg.norm(gv - self.vis) / torch.linalg.norm(self.vis)
        return {"image_err_vs_exact_dft": float("%.3g" % e_i.item()),
                "vis_err_vs_exact_dft": float("%.3g" % e_v.item())}


def wstack_form(_lib, torch, d, u, v, w, V, W, model, steps, exact):
    """W-stacking hybrid (Section 4.3) on the array-scale workload: 16 uniform
    w-slices over the same w range, 8 residual planes per slice (the plain
    path's plane density), grid (x n) + degrid (/ n) per step; then 16
    density-adapted slices; for each, the errors of sampled pixels and
    predictions against the exact DFT."""
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
    res.update(exact.errors(torch, img, vis_out))
    ws.close()
    K.close()
    # the same number of slices with density-adapted edges (about equal
    # counts: narrow near w = 0, wide at large |w|), each slice with residual
    # tables on its own range (the kernels' w range is not used)
    edges = _lib.density_edges(w, ns, d["w_lo"], d["w_hi"])
    K = _lib.Kernels(N, fov, S, O, P, d["w_lo"], d["w_hi"])
    t = time.perf_counter()
    ws = _lib.WStack(K, ns, 0.0, 0.0, u, v, w, edges=edges)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t
    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    widths = edges[1:] - edges[:-1]
    res["density_edges"] = {
        "ms_per_step": round(ms, 3), "Mvis_per_s": round(ws.nvis / (ms * 1e-3) / 1e6, 2),
        "narrowest_slice": round(float(min(widths)), 1), "widest_slice": round(float(max(widths)), 1),
        "create_s": round(t_create, 3),
        **exact.errors(torch, img, vis_out)}
    ws.close()
    K.close()
    return res


def correction_form(_lib, torch, d, u, v, w, V, W, model, steps, Sc=13, Oc=8):
    """The correction table F_w - F~_w (Section 6) attached to the array-scale
    kernels (S_c = 13, O_c = 8): its FP64 generation for the 128 planes (and
    its factoring into separable terms), then grid (x n) + degrid (/ n) per
    step with the correction run as those terms on the matrix-core kernels;
    then the same step with the passes that walk the table, and the relative
    difference of the two forms' images and visibilities."""
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
           "table_generation_ms": round(table_ms, 2), "separable_terms": K.correction_rank(),
           "ms_per_step": round(ms, 3), "Mvis_per_s": round(plan.nvis / (ms * 1e-3) / 1e6, 2),
           "stages_ms_per_step": {k: round(v_ / steps, 4) for k, (v_, n) in st.items() if n}}
    img_t, vis_t = img.clone(), vis_out.clone()
    K.correction_terms(False)
    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms_w = (time.perf_counter() - t0) * 1e3 / steps
    res["table_walk"] = {
        "ms_per_step": round(ms_w, 3),
        "rel_diff_terms_vs_walk": {"image_inner_half": rel_diff(torch, img_t, img, inner=True),
                                   "vis": rel_diff(torch, vis_t, vis_out)}}
    plan.close()
    K.close()
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


def wsnap_form(_lib, torch, d, u, v, w, V, W, model, steps, exact, n_snap=16, planes=16):
    """W snapshots (Section 4.2) on the array-scale workload: 16 snapshots of
    30 min (contiguous in the time-ordered data), a plane fitted per snapshot,
    16 residual planes, grid (x n) + degrid (/ n) per step; plus the errors
    of sampled pixels and predictions against the exact DFT."""
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
    res.update(exact.errors(torch, img, vis_out))
    ws.close()
    K.close()
    return res


def differentiation_form(_lib, torch, steps):
    """The differentiation workload: a 2048^2 real model, 4,285,440 visibilities
    (32 antennas, 4 km, 6 h in 20 s dumps, 8 channels), 64 planes, S = 15:
    V_t = A x_true + complex noise of 0.1 rms(A x_true); one step is
    chi^2(Predict(x)) and its gradient (degrid forward, gridding adjoint
    backward) at x = 0.9 x_true."""
    import numpy as np

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
            item_slots(2048)   # per-facet launches with the default work-item length
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
    ap.add_argument("--forms", choices=("all", "precision", "none"), default="all",
                    help="forms measured beside the FP32 step: all, only the FP16/BF16 "
                         "MFMA forms, or none")
    ap.add_argument("--fp32-only", action="store_true", help="same as --forms none")
    ap.add_argument("--no-weights", action="store_true",
                    help="pass W = NULL (unit weights implied) instead of an array of ones")
    args = ap.parse_args()
    if args.fp32_only:
        args.forms = "none"

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
    # model image for the prediction: complex Gaussian on the inner half, 0
    # outside (where 1 / (c1 c1) would amplify it by up to ~1e7)
    g = torch.Generator(device="cuda").manual_seed(1511)
    model = torch.zeros((N, N), dtype=torch.complex64, device="cuda")
    model[N // 4:3 * N // 4, N // 4:3 * N // 4] = torch.randn(
        (N // 2, N // 2), dtype=torch.complex64, device="cuda", generator=g)
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
    ref_img, ref_vis = img.clone(), vis_out.clone()   # outputs of the last FP32 step
    t = time.perf_counter()
    exact = ExactDFT(torch, d, u, v, w, V, W, model)
    accuracy = exact.errors(torch, ref_img, ref_vis)
    log("exact references in %.1f s; FP32 step: %s" % (time.perf_counter() - t, accuracy))

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
    if args.forms != "none":
        for prec in ("fp16", "bf16"):
            ms, st, _ = measure(prec)
            # errors of this step's outputs relative to the FP32 step's, on
            # the same array-scale data (FP32 is within 1e-6 of the FP64
            # reference there, so these are the 16-bit forms' own errors)
            g_ms = st["grid"][0] / max(st["grid"][1], 1)
            d_ms = st["degrid"][0] / max(st["degrid"][1], 1)
            forms[prec] = {"value": round(nvis / (ms * 1e-3) / 1e6, 2), "ms_per_step": round(ms, 3),
                           "grid_ms": round(g_ms, 4), "degrid_ms": round(d_ms, 4),
                           # grid + degrid kernel time of the FP32 step over this form's
                           "kernels_speedup_vs_fp32": round(
                               (per_launch["grid"] + per_launch["degrid"]) / (g_ms + d_ms), 3),
                           "rel_rms_err_vs_fp32": {
                               "image_inner_half": rel_diff(torch, img, ref_img, inner=True),
                               "image_full": rel_diff(torch, img, ref_img),
                               "vis": rel_diff(torch, vis_out, ref_vis)},
                           **exact.errors(torch, img, vis_out)}
            log("%s: %s" % (prec, forms[prec]))

    if args.forms == "all":
        forms["batched_facets"] = batching_form(_lib, torch, args)
        forms["w_stacking"] = wstack_form(_lib, torch, d, u, v, w, V, W, model, min(args.steps, 5),
                                          exact)
        log("w-stacking: %s" % forms["w_stacking"])
        forms["correction_table"] = correction_form(_lib, torch, d, u, v, w, V, W, model,
                                                    min(args.steps, 5))
        log("correction table: %s" % forms["correction_table"])
        forms["channel_shared"] = channel_form(_lib, torch, d, u, v, w, V, W, model, args.steps)
        log("channel-shared coordinates: %s" % forms["channel_shared"])
        forms["w_snapshots"] = wsnap_form(_lib, torch, d, u, v, w, V, W, model, min(args.steps, 5),
                                         exact)
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
        # the FP32 step's sampled outputs against the exact DFT (FP64)
        "accuracy": accuracy,
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
