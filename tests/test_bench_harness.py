"""bench.py's host-side pieces, without a GPU: the one-GPU guard, the HBM
traffic reader (numbers only while the kernels' sources are unchanged) and the
exact-DFT references of its accuracy fields, checked against the oracle's
direct DFT on a small case."""
import hashlib
import importlib.util
import json
import math
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_traffic_reported_only_for_unchanged_sources(bench, tmp_path, monkeypatch):
    text = open(bench.TRAFFIC_FILE).read()
    block = json.loads(text.split("```json\n")[1].split("\n```")[0])
    for k in ("grid", "degrid"):
        e = block["kernels"][k]
        h = hashlib.sha256()
        for src in e["sources"]:
            h.update(open(os.path.join(ROOT, src), "rb").read())
        want = e["bytes_per_launch"] if h.hexdigest() == e["sources_sha256"] else None
        assert bench.measured_traffic(k) == want
        assert e["bytes_per_launch"] > e["algorithmic_bytes"]
        e["sources_sha256"] = h.hexdigest()      # as if just measured
    block["kernels"]["degrid"]["sources_sha256"] = "0" * 64
    f = tmp_path / "traffic.md"
    f.write_text("```json\n" + json.dumps(block) + "\n```\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("degrid") is None
    assert bench.measured_traffic("grid") == block["kernels"]["grid"]["bytes_per_launch"]
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.md"))
    assert bench.measured_traffic("grid") is None


def test_exact_references_match_the_oracle_dft(bench):
    torch = pytest.importorskip("torch")
    N, fov = 32, math.radians(3.0)
    rng = np.random.default_rng(1)
    n = 500
    u = rng.uniform(-12, 12, n) / fov
    v = rng.uniform(-12, 12, n) / fov
    w = rng.uniform(-300, 300, n)
    V = (rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(np.complex64)
    W = rng.uniform(0.5, 2, n).astype(np.float32)
    X = np.zeros((N, N), np.complex64)
    X[8:24, 8:24] = rng.standard_normal((16, 16))
    t = lambda a, dt: torch.as_tensor(a, dtype=dt)  # noqa: E731
    ex = bench.ExactDFT(torch, dict(N=N, fov=fov), t(u, torch.float64), t(v, torch.float64),
                        t(w, torch.float64), t(V, torch.complex64), t(W, torch.float32),
                        t(X, torch.complex64), npix=16, nv=32)
    exact = oracle.dft.phase_screen(N, fov, "exact")
    l = (np.arange(N) - N / 2) * fov / N
    nn = np.sqrt(1 - l[None, :] ** 2 - l[:, None] ** 2)
    D = nn * oracle.dft.dirty(u, v, w, V.astype(complex) * W, N, fov, exact)
    ref = D[ex.pq[1], ex.pq[0]]
    assert np.max(np.abs(ex.image.numpy() - ref)) <= 1e-12 * np.max(np.abs(ref))
    vi = ex.vi.numpy()
    P = oracle.dft.predict(u[vi], v[vi], w[vi], X.astype(complex) / nn, N, fov, exact)
    assert np.max(np.abs(ex.vis.numpy() - P)) <= 1e-12 * np.max(np.abs(P))
    # errors of the references themselves are zero, of a perturbed image not
    img = torch.zeros((N, N), dtype=torch.complex128)
    img[ex.pq[1], ex.pq[0]] = ex.image
    vis = torch.zeros(n, dtype=torch.complex128)
    vis[ex.vi] = ex.vis
    e = ex.errors(torch, img, vis)
    assert e["image_err_vs_exact_dft"] == 0.0 and e["vis_err_vs_exact_dft"] == 0.0
    e = ex.errors(torch, img * 1.01, vis)
    assert e["image_err_vs_exact_dft"] == pytest.approx(0.01, rel=1e-6)
