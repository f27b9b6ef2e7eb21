"""Host logic of bench.py: recorded counter figures are used only for the
kernel and the kernel sources they were taken from, and the derived
ceilings follow from the recorded counts and the launch time."""
import os
import shutil

import pytest

import bench


def _copy_sources(tmp_path):
    for rel in bench.KERNEL_SOURCES:
        dst = tmp_path / rel
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(bench.ROOT, rel), dst)


def test_recorded_figures_are_gated_on_kernel_and_sources(monkeypatch, tmp_path):
    """A counter summary is used only for the kernel it names and only while
    the kernel sources hash to the recorded value."""
    _copy_sources(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    kernel = "k_migrate_tile<3,false>"
    summary = tmp_path / bench.TRAFFIC_FILE
    summary.parent.mkdir(parents=True, exist_ok=True)
    summary.write_text("# summary\n\n- kernel: `%s`\n- fetch_bytes_per_launch: 1000\n"
                       "- write_bytes_per_launch: 500\n- kernel_sources_sha256: %s\n"
                       % (kernel, bench.kernel_sources_sha256()))
    t = bench.recorded_traffic(kernel)
    assert t is not None and t["bytes_per_launch"] == 1500
    assert bench.recorded_traffic("k_migrate_wave<3,false>") is None
    # any change to a kernel source voids the recorded figures
    src = tmp_path / bench.KERNEL_SOURCES[0]
    src.write_text(src.read_text() + "\n// edited\n")
    assert bench.recorded_traffic(kernel) is None
    assert bench.recorded_valu(kernel, 4e-4) is None


def test_valu_figures_arithmetic():
    rec = {"sq_insts_valu_per_launch": "6144", "sq_insts_valu_add_f64_per_launch": "10",
           "sq_insts_valu_mul_f64_per_launch": "20", "sq_insts_valu_fma_f64_per_launch": "30",
           "sq_insts_valu_trans_f64_per_launch": "5", "sq_insts_lds_per_launch": "7",
           "sq_insts_vmem_rd_per_launch": "3"}
    f = bench._valu_figures(rec, 1e-6)
    assert f["issue_rate"] == pytest.approx(6144 / 1e-6)
    # 256 CUs x 4 SIMDs x 2.4 GHz, one wave64 VALU instruction per 4 cycles
    assert f["issue_frac"] == pytest.approx(6144 / 1e-6 / (256 * 4 * 2.4e9 / 4))
    assert f["fp64_insts_per_launch"] == 65
    # FMA counts two operations, every instruction all 64 lanes
    assert f["fp64_lane_tflops_upper"] == pytest.approx(64 * (10 + 20 + 5 + 60) / 1e-6 / 1e12)


def test_more_than_one_gpu_is_refused():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and not r.stdout.strip()
