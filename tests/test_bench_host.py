"""Host-side logic of bench.py (CPU only): the roofline arithmetic, the
gating of the stored HBM-traffic figure on the kernel source, and the refusal
to run on more than one GPU."""
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    sys.path.insert(0, ROOT)
    import bench as B
    return B


def fake_md(kt, T=3, F=128, K=20, n=24000, edges=1_000_000.0):
    return {"hdr": {"F": F, "K": K, "T": T}, "n": n, "kt": kt, "n_edges_mean": edges}


def test_roofline_over_the_layers_after_the_first(bench):
    # 10 steps, 2 adjoint launches per step of 0.5 ms each: the first layer is
    # factorised and not among the timed launches
    steps = 10
    kt = {"msg_fwd": (3.0, 20), "msg_bwd": (10.0, 20)}
    r = bench.roofline(fake_md(kt), "bf16", steps)
    later = bench.per_edge_flops(128, 20)["msg_bwd"][1]
    assert r["kernel"] == "msg_bwd" and r["bound"] == "mfma"
    assert r["avg_launch_us"] == pytest.approx(500.0)
    assert r["achieved"] == pytest.approx(later * 1e6 / 500e-6 / 1e12, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / 2500.0, rel=1e-3)
    assert "after the first" in r["work_per_launch"]


def test_roofline_over_every_layer(bench):
    # 3 launches per step: the first layer's work enters the average
    steps = 10
    kt = {"msg_fwd": (3.0, 30), "msg_bwd": (15.0, 30)}
    r = bench.roofline(fake_md(kt), "fp32", steps)
    first, later = bench.per_edge_flops(128, 20)["msg_bwd"]
    assert r["achieved"] == pytest.approx((first + 2 * later) / 3 * 1e6 / 500e-6 / 1e12, rel=1e-3)
    assert r["peak"] == pytest.approx(157.3)


def test_per_edge_flops_counts(bench):
    # one filter output is K + 1 multiply-adds (2 flops each)
    pe = bench.per_edge_flops(128, 20)
    assert pe["msg_fwd"] == (4 * 21 * 128 + 9 * 128, 6 * 21 * 128 + 16 * 128)
    assert pe["msg_bwd"] == (6 * 21 * 128 + 18 * 128, 12 * 21 * 128 + 39 * 128)


def test_traffic_figure_is_gated_on_the_kernel_source(bench, tmp_path, monkeypatch):
    src = os.path.join(ROOT, "profiles", "traffic_msg_bwd_bf16.json")
    d = json.load(open(src))
    (tmp_path / "profiles").mkdir()
    (tmp_path / "paper_2506_04055_amd" / "csrc").mkdir(parents=True)
    shutil.copy(os.path.join(ROOT, "paper_2506_04055_amd", "csrc", "msg.hip"),
                tmp_path / "paper_2506_04055_amd" / "csrc" / "msg.hip")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    dst = tmp_path / "profiles" / "traffic_msg_bwd_bf16.json"
    # the stored hash of the current source: the figure is used
    d_ok = dict(d, source_sha256_16=bench.source_hash("msg.hip"))
    dst.write_text(json.dumps(d_ok))
    assert bench.load_traffic("msg_bwd", "bf16") == d["hbm_bytes_per_launch"]
    # any other source: the figure is withheld
    dst.write_text(json.dumps(dict(d, source_sha256_16="0" * 16)))
    assert bench.load_traffic("msg_bwd", "bf16") is None
    # no file: withheld
    dst.unlink()
    assert bench.load_traffic("msg_bwd", "bf16") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
