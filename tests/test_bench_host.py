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


def fake_stats(T=3):
    # hop sets of a domain share: atoms and pruned in-edges within <= h hops
    return {"n_within_hops": [1000, 1100, 1200, 1300] + [0] * 4,
            "n_edges_within_hops": [35000, 38500, 42000, 45500] + [0] * 4}


def test_layer_work_follows_the_hop_sets(bench):
    w = bench.layer_work(fake_stats(), 3, factorised=True)
    # forward layer t reaches destinations within T-1-t hops, the adjoint of
    # layer t the sources within T-t hops; the factorised first layer is absent
    assert w["msg_fwd"] == [(1, 38500, 1100), (2, 35000, 1000)]
    assert w["msg_bwd"] == [(2, 38500, 1100), (1, 42000, 1200)]
    w = bench.layer_work(fake_stats(), 3, factorised=False)
    assert w["msg_fwd"][0] == (0, 42000, 1200) and w["msg_bwd"][-1] == (0, 45500, 1300)


def test_roofline_entry_picks_the_binding_roof(bench):
    F, K = 128, 20
    work = bench.layer_work(fake_stats(), 3, factorised=True)["msg_bwd"]
    later = bench.per_edge_flops(F, K)["msg_bwd"][1]
    eb, ab = bench.per_pass_bytes(F)["msg_bwd"]
    flops = (later * 38500 + later * 42000) / 2
    byts = (eb * 38500 + ab * 1100 + eb * 42000 + ab * 1200) / 2
    avg = 1e-4
    # split bf16: bytes / 8 TB/s exceed flops / 2.5 PF, so HBM binds
    r = bench.roofline_entry("msg_bwd", work, F, K, avg, "bf16", "fcc1m")
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(byts / avg / 1e9, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0, rel=1e-3)
    assert r["other_roof"]["achieved"] == pytest.approx(flops / avg / 1e12, rel=1e-3)
    # FP32 filter: the matrix cores' FP32 rate binds
    r = bench.roofline_entry("msg_bwd", work, F, K, avg, "fp32", "fcc1m")
    assert r["bound"] == "mfma" and r["peak"] == pytest.approx(157.3)
    assert r["achieved"] == pytest.approx(flops / avg / 1e12, rel=1e-3)
    # the bf16-node form keeps the filter in FP32: same roof as fp32
    assert bench.roofline_entry("msg_bwd", work, F, K, avg, "bf16_node", "fcc1m")["bound"] == "mfma"


def test_per_edge_counts(bench):
    pe = bench.per_edge_flops(128, 20)
    assert pe["msg_fwd"][1] == 6 * 20 * 128 + 12 * 128
    assert pe["msg_bwd"][1] == 12 * 20 * 128 + 28 * 128
    assert bench.per_pass_bytes(128)["msg_bwd"] == (36, 19 * 128 * 4 + 8)


def test_node_flops_with_active_sets(bench):
    hops = [1000, 1100, 1200, 1300]
    F, T = 128, 3
    f = bench.node_flops_per_step(hops, F, T, 1000)
    fwd = 22 * F * F * 1200 + (8 * F * F * 1200 + 22 * F * F * 1100) + (8 * F * F * 1100 + 22 * F * F * 1000)
    assert f == 2 * fwd + 2 * F * F * 1000


def test_traffic_figure_is_gated_on_the_kernel_source(bench, tmp_path, monkeypatch):
    d = {"kernel": "msg_bwd", "precision": "bf16", "hbm_bytes_per_launch": 123456789}
    (tmp_path / "profiles").mkdir()
    (tmp_path / "paper_2506_04055_amd" / "csrc").mkdir(parents=True)
    for f in ("msg.hip", "nbr.hip"):
        shutil.copy(os.path.join(ROOT, "paper_2506_04055_amd", "csrc", f), tmp_path / "paper_2506_04055_amd" / "csrc" / f)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    dst = tmp_path / "profiles" / "traffic_msg_bwd_fcc1m_bf16.json"
    # the stored hashes of the current sources: the figure is used
    ok = {"msg.hip": bench.source_hash("msg.hip"), "nbr.hip": bench.source_hash("nbr.hip")}
    dst.write_text(json.dumps(dict(d, source_sha256_16=ok)))
    assert bench.load_traffic("msg_bwd", "bf16", "fcc1m") == d["hbm_bytes_per_launch"]
    # the kernel or the atom order changed since: the figure is withheld
    for f in ok:
        dst.write_text(json.dumps(dict(d, source_sha256_16=dict(ok, **{f: "0" * 16}))))
        assert bench.load_traffic("msg_bwd", "bf16", "fcc1m") is None
    # a single hash (the old form) or no file: withheld
    dst.write_text(json.dumps(dict(d, source_sha256_16=ok["msg.hip"])))
    assert bench.load_traffic("msg_bwd", "bf16", "fcc1m") is None
    dst.unlink()
    assert bench.load_traffic("msg_bwd", "bf16", "fcc1m") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
