"""Host-side checks that need no GPU: the benchmark's one-GPU contract and
the determinism of the seeded input generators."""
import json
import os
import subprocess
import sys

import numpy as np

import scenegen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_scene_independent_of_thread_count(monkeypatch):
    a = scenegen.make_scene(scenegen.TINY)
    monkeypatch.setattr(scenegen, "_threads", lambda: 1)
    b = scenegen.make_scene(scenegen.TINY)
    for k in ("grid", "plane_xy", "plane_xz", "plane_yz", "occ", "mlp"):
        assert np.array_equal(a[k], b[k]), k


def test_ray_orders_are_permutations():
    for order in ("row", "tile4", "morton"):
        p = scenegen.pixel_order(64, 48, order)
        assert np.array_equal(np.sort(p), np.arange(64 * 48)), order
    # a 4x4 tile / Morton block of 16 consecutive rays is a 4x4 pixel square
    for order in ("tile4", "morton"):
        p = scenegen.pixel_order(64, 48, order)[:16]
        ys, xs = np.divmod(p, 64)
        assert ys.max() - ys.min() == 3 and xs.max() - xs.min() == 3


def test_towers_scene_has_uneven_intervals():
    cfg = scenegen.SceneConfig(grid=(8, 8, 8), planes=(8, 8, 8), occ=64, band=0.01, tower_fraction=0.1)
    sc = scenegen.make_scene(cfg)
    thick = sc["occ"][..., 1] - sc["occ"][..., 0]
    assert (thick > 0.019).mean() >= 0.1
    assert thick.max() <= 0.25 + 1e-6


def test_traffic_figure_only_for_the_profiled_kernel_source(tmp_path, monkeypatch):
    """The bench reports the committed HBM traffic only while the hashed
    kernel sources are the ones the counters were taken on."""
    import shutil

    sys.path.insert(0, ROOT)
    import bench

    csrc = tmp_path / "paper_2404_09531_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in bench.KERNEL_SOURCES["fwd"]:
        shutil.copy(os.path.join(ROOT, "paper_2404_09531_amd", "csrc", f), csrc / f)
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("k", "w") is None  # no record file
    rec = {"k": {"w": {"source_hash": bench.kernel_source_hash(), "hbm_bytes_per_launch": 1234}}}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    assert bench.measured_traffic("k", "w") == 1234
    assert bench.measured_traffic("k", "other") is None
    with open(csrc / "march_fwd.hip", "a") as fh:
        fh.write("\n// edited\n")
    assert bench.measured_traffic("k", "w") is None


def test_oracle_pool_equals_serial_oracle():
    """render_parallel splits the rays over worker processes and returns what
    oracle_render returns; the k-list check flags exactly the altered rays."""
    import numpy as np

    import oracle
    import scenegen
    from oracle.parallel import render_parallel

    sc = scenegen.make_scene(scenegen.TINY)
    o, d = scenegen.oblique_rays(300, seed=5)
    prm = oracle.RenderParams(n_max=64, c_bg=(0.25, 0.5, 0.75))
    ref = oracle.oracle_render(sc, o, d, prm)
    k = ref["k_list"].copy()
    k[7, 0] += 1
    k[250, 3] = -5
    par = render_parallel(sc, o, d, prm, workers=2, chunk=64, k_list=k)
    for key in ("C", "T", "F", "n_placed", "n_eval"):
        assert np.array_equal(par[key], ref[key]), key
    assert par["k_mismatch_rays"].tolist() == [7, 250]
    assert par["workers"] == 2


def test_calibration_library_refuses_bad_shapes_before_launching():
    """The bench's calibration kernels (libomcalib.so) check their arguments
    on the host and return -1 without launching anything: no GPU is needed
    to see a refusal."""
    import ctypes

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    lib = ctypes.CDLL(os.path.join(root, "paper_2404_09531_amd", "libomcalib.so"))
    lib.omcalib_atomic_segments.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_void_p]
    lib.omcalib_l1_gather.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_void_p, ctypes.c_void_p]
    fake = 1 << 20
    for nseg, blocks, iters in ((3, 1, 1), (0, 1, 1), (1 << 27, 1, 1), (1 << 10, 0, 1), (1 << 10, 1, 0)):
        assert lib.omcalib_atomic_segments(fake, nseg, blocks, iters, None) == -1
    assert lib.omcalib_atomic_segments(None, 1 << 10, 1, 1, None) == -1
    for nvec, span in ((1000, 4), (8, 4), (1024, 3), (1024, 32)):
        assert lib.omcalib_l1_gather(fake, nvec, span, 1, 1, fake, None) == -1


def _counter_csv(path, rows):
    """A rocprofv3-style counter CSV: (dispatch id, kernel name, counter, value)."""
    path.parent.mkdir(parents=True, exist_ok=True)
    lines = ["Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value"]
    lines += [f'{i},"{k}",{c},{v}' for i, k, c, v in rows]
    path.write_text("\n".join(lines) + "\n")


def test_traffic_summary_scales_by_the_copy_calibration(tmp_path, monkeypatch):
    """bench_counters.py traffic: the per-launch DRAM bytes are the median
    FETCH_SIZE and WRITE_SIZE of the kernel's dispatches (KiB), each scaled
    by what the counter reads for the 1 GiB copy of the same run; --slice
    selects dispatches; a pattern must name exactly one kernel."""
    import argparse

    import pytest

    sys.path.insert(0, ROOT)
    import bench_counters as bc

    copy = "__amd_rocclr_copyBuffer"
    kern = "void omerf::k_march_fwd_f32q<false, false, false>(omerf::SceneDev)"
    other = "void omerf::k_march_fwd_f32q<true, false, false>(omerf::SceneDev)"
    # the copy reads 2^30 B and writes 2^30 B: FETCH_SIZE counts half of it
    _counter_csv(tmp_path / "f" / "x_counter_collection.csv",
                 [(0, copy, "FETCH_SIZE", 524288.0), (9, other, "FETCH_SIZE", 7.0)] +
                 [(i + 1, kern, "FETCH_SIZE", v) for i, v in enumerate((100.0, 300.0, 500.0))])
    _counter_csv(tmp_path / "w" / "x_counter_collection.csv",
                 [(0, copy, "WRITE_SIZE", 1048576.0), (9, other, "WRITE_SIZE", 7.0)] +
                 [(i + 1, kern, "WRITE_SIZE", v) for i, v in enumerate((10.0, 30.0, 50.0))])
    rec_path = tmp_path / "traffic.json"
    monkeypatch.setattr(bc, "TRAFFIC", str(rec_path))
    monkeypatch.setattr(bc, "source_hash", lambda fam: "h-" + fam)

    def run(workload, slc, spec):
        bc.cmd_traffic(argparse.Namespace(fetch=str(tmp_path / "f"), write=str(tmp_path / "w"), workload=workload,
                                          slice=slc, kernels=[spec]))
        return json.loads(rec_path.read_text())

    rec = run("all", None, "k=k_march_fwd_f32q<false")
    e = rec["k"]["all"]
    assert e["fetch_scale"] == 2.0 and e["write_scale"] == 1.0
    assert e["hbm_bytes_per_launch"] == 300 * 1024 * 2 + 30 * 1024  # medians of the three dispatches
    assert e["dispatches"] == 3 and e["source_hash"] == "h-fwd"
    rec = run("first-two", "0:2", "k=k_march_fwd_f32q<false")
    assert rec["k"]["first-two"]["hbm_bytes_per_launch"] == 200 * 1024 * 2 + 20 * 1024
    assert rec["k"]["all"]["hbm_bytes_per_launch"] == 300 * 1024 * 2 + 30 * 1024  # kept
    with pytest.raises(SystemExit):
        run("none", None, "k=k_mlp_bwd")        # no such kernel
    with pytest.raises(SystemExit):
        run("many", None, "k=k_march_fwd_f32q")  # two kernels match


def test_counter_summary_takes_medians_and_mfma_fraction(tmp_path, monkeypatch):
    """bench_counters.py counters: per counter the median over the kernel's
    dispatches, recorded with the hash of its source family; rocprofv3's
    MfmaUtil (percent) also becomes the fraction the bench reports."""
    import argparse

    sys.path.insert(0, ROOT)
    import bench_counters as bc

    kern = "void omerf::k_mlp_bf16<10>(float const*)"
    rows = [(i, kern, "MfmaUtil", v) for i, v in enumerate((6.0, 7.0, 9.0))]
    rows += [(i + 3, kern, "TCC_ATOMIC_sum", v) for i, v in enumerate((5.0, 1.0, 3.0))]
    _counter_csv(tmp_path / "c" / "y_counter_collection.csv", rows)
    rec_path = tmp_path / "traffic.json"
    monkeypatch.setattr(bc, "TRAFFIC", str(rec_path))
    monkeypatch.setattr(bc, "source_hash", lambda fam: "h-" + fam)
    bc.cmd_counters(argparse.Namespace(dir=str(tmp_path / "c"), workload="w", kernels=["k_mlp_bf16<10>=k_mlp_bf16<10>"]))
    e = json.loads(rec_path.read_text())["k_mlp_bf16<10>"]["w"]
    assert e["counters"] == {"MfmaUtil": 7.0, "TCC_ATOMIC_sum": 3.0}
    assert e["mfma_busy_frac"] == 0.07
    assert e["family"] == "mlp" and e["counter_source_hash"] == "h-mlp" and e["source_hash"] == "h-mlp"
