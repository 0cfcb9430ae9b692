"""Host-side logic of bench.py (no GPU): the source fingerprint that keys measured HBM
traffic, the workload description under --nz, and the algorithmic work count."""
import math
import os
import shutil

import bench

CSRC = ("ssp_device.hip", "ssp_device.h", "ssp_tuned.h")


def _copy_sources(tmp_path):
    dst = tmp_path / "paper_2511_03343_amd" / "csrc"
    dst.mkdir(parents=True)
    for f in CSRC:
        shutil.copy(os.path.join(bench.ROOT, "paper_2511_03343_amd", "csrc", f), dst / f)
    return dst


def test_fingerprint_ignores_comments_and_blank_lines(tmp_path):
    dst = _copy_sources(tmp_path)
    base = bench.source_fingerprint(str(tmp_path))
    assert base == bench.source_fingerprint()
    with open(dst / "ssp_device.hip", "a") as fh:
        fh.write("\n// a note\n/* a block\n   comment */\n\n")
    assert bench.source_fingerprint(str(tmp_path)) == base


def test_fingerprint_changes_with_code(tmp_path):
    dst = _copy_sources(tmp_path)
    base = bench.source_fingerprint(str(tmp_path))
    text = (dst / "ssp_tuned.h").read_text()
    (dst / "ssp_tuned.h").write_text(text.replace("kTunedVariant[9] = {0", "kTunedVariant[9] = {1", 1))
    assert bench.source_fingerprint(str(tmp_path)) != base


def test_measured_traffic_is_keyed_by_grid_and_boundary():
    key = next(iter(bench.TRAFFIC))
    workload, nz, batch, chunk = key
    assert bench.measured_traffic(workload, nz + 1, batch, chunk) is None
    assert bench.measured_traffic(workload, nz, batch, chunk, "periodic") is None


def test_measured_traffic_belongs_to_the_current_sources():
    # the counter figures in bench.py were taken on the kernels of this tree: the dominant
    # kernels of the default line (the broadband split group) and of its munk4096 and
    # eddy16384 keys
    assert set(bench.TRAFFIC) >= {("broadband", 32768, 150, 40), ("munk4096", 4096, 512, 100),
                                  ("eddy16384", 16384, 256, 50)}
    fp = bench.source_fingerprint()
    for key, t in bench.TRAFFIC.items():
        assert t["fingerprint"] == fp, key
        assert bench.measured_traffic(*key) == t["fetch"] + t["write"] > 0


def test_workload_description_names_the_grid():
    assert "Nz=4095" in bench._describe("munk4096", 4095)
    assert "Nz=4096" in bench._describe("munk4096", None)
    assert "Nz=8191" in bench._describe("broadband", 8191)


def test_algorithmic_flops_count():
    # two DSTs of 5 Nz log2 Nz plus 8 Nz per Neumann term, 16 Nz per Pade factor and step,
    # one DST per output
    nz, p, terms, steps, outputs = 4096, 6, 10, 3, 2
    tr = 5 * nz * math.log2(nz)
    want = terms * 2 * (tr + 8 * nz) + steps * p * 16 * nz + outputs * tr
    assert bench.algorithmic_flops(nz, p, terms, steps, outputs) == want


def test_more_than_one_gpu_is_refused_with_a_message():
    # every solve is independent; the benchmark measures one GPU and says so for N > 1
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout.strip() == ""
