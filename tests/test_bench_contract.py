"""CPU checks of the benchmark's contract: the algorithmic byte count behind the roofline
figure, the traffic record's source gate, and the refusal of more than one GPU."""
import hashlib
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_algorithmic_bytes_of_the_headline_apply():
    # Q4 (P = Q = 5) on 34^3 elements: (34*4+1)^3 nodes; per apply the 16-scalar state
    # once, du read and y written once, the int32 element map once
    E, P, Q, N = 34 ** 3, 5, 5, (34 * 4 + 1) ** 3
    assert N == 2_571_353
    state = E * Q ** 3 * 16 * 8
    vectors = 2 * 3 * N * 8
    emap = 4 * E * P ** 3
    assert bench.algorithmic_bytes(E, P, Q, N, 8) == state + vectors + emap == 771_940_944
    # the FP32 apply moves half the state and vector bytes, the same map
    assert bench.algorithmic_bytes(E, P, Q, N, 4) == state // 2 + vectors // 2 + emap


def test_traffic_record_is_gated_by_the_kernel_source():
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic_jacobian_q4_fp64_34cubed.json")))
    src = open(os.path.join(ROOT, "paper_2204_01722_amd", "csrc", "op_kernels.hip"), "rb").read()
    current = rec["source_sha256"] == hashlib.sha256(src).hexdigest()
    assert (bench.measured_traffic() is not None) == current
    if current:
        assert rec["bytes_per_apply"] >= rec["algorithmic_bytes_per_apply"] == 771_940_944


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=300)
    assert res.returncode == 2
    assert "one GPU" in res.stderr


def test_jsonl_log_appends_one_record_per_run(tmp_path):
    path = str(tmp_path / "runs.jsonl")
    rec = {"metric": "m", "value": 1.5, "roofline": {"frac": 0.5}}
    bench.append_jsonl(path, rec, {"steps": 20, "warmup": 5})
    bench.append_jsonl(path, dict(rec, value=2.5), {"steps": 10, "warmup": 2})
    lines = [json.loads(x) for x in open(path).read().splitlines()]
    assert [x["value"] for x in lines] == [1.5, 2.5]
    assert lines[0]["roofline"] == {"frac": 0.5} and lines[1]["run"]["args"] == {"steps": 10, "warmup": 2}
    assert lines[0]["run"]["host_cpus"] == os.cpu_count() and "time" in lines[0]["run"]
    assert "run" not in rec  # the printed record is left as it is
