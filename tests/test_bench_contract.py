"""CPU checks of the benchmark script and the committed profile summaries:
the one-GPU contract of bench.py, the byte counters it reports being taken
at the current kernel sources, and every profile summary naming the kernel
source it was taken at and a command that runs committed files."""
import glob
import hashlib
import json
import os
import re
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_counters_match_current_kernel_sources():
    # bench.py reports traffic only while these hold; a kernel change must
    # come with counters taken again
    assert bench.kernel_source_hash("gemm.hip", bench.GEMM_STEP_END) == bench.COUNTERS["kernel_source_sha256_16"]
    assert bench.kernel_source_hash("gemm.hip", bench.GEMM_STEP_END) == bench.COUNTERS_HBM["kernel_source_sha256_16"]
    assert bench.COUNTERS_HBM["cfg"] == bench.HBM_CFG  # taken on the tile shape the HBM point pins
    assert (bench.kernel_source_hash("factored.hip", bench.FACT_DEVICE_END)
            == bench.COUNTERS_FACT["kernel_source_sha256_16"])


def test_profiles_name_their_source_and_a_committed_command():
    files = sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md")))
    assert files
    for path in files:
        text = open(path).read()
        name = os.path.basename(path)
        cmds = [l.strip() for l in text.splitlines() if l.strip().startswith("rocprofv3 ")]
        assert cmds, f"{name}: no rocprofv3 command"
        for c in cmds:
            assert "_work" not in c and "/root/reference" not in c, f"{name}: {c}"
            prog = c.split(" -- ", 1)[1].split()
            assert prog[0] in ("python3", "python"), f"{name}: {c}"
            for arg in prog[1:]:
                if arg.endswith(".py") or arg.startswith("tests/"):
                    assert os.path.exists(os.path.join(ROOT, arg.split("::")[0])), f"{name}: {arg}"
        # a stated kernel-source hash is that of the source as committed (the
        # part before the file's marker, where the profile says "(text before")
        for m in re.finditer(r"(\(text before[^`]*)?sha256\[:16\] of\s+`([^`]+)`:\s+`([0-9a-f]{16})`", text):
            data = open(os.path.join(ROOT, m.group(2)), "rb").read()
            if m.group(1):
                data = data[:data.index(bench.SOURCE_MARKERS[os.path.basename(m.group(2))])]
            assert hashlib.sha256(data).hexdigest()[:16] == m.group(3), f"{name}: {m.group(2)} changed"
        if name.startswith("density_kernel"):
            assert "csrc/grid.hip`: `" in text, f"{name}: grid.hip hash not stated"
