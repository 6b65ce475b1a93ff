"""CPU checks of bench.py's host logic: the single-GPU refusal, the hash that ties
committed hardware-counter summaries to the gather kernel's code, and the lookup
that reports HBM traffic only for counters taken on the same kernel, tile and
launch size."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

KERNEL = """// gather
template <typename WT, int K>
__global__ void k_pull(int t, const float *w, float *out) {
    // every row
    out[t] += w[t];  /* one add */
}
"""
DEVICE = "// helpers\n__device__ int lane_id() { return threadIdx.x & 63; }\n"


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr + r.stdout


def test_source_hash_ignores_comments_and_blank_lines():
    base = bench.kernel_source_sha("pull", KERNEL, DEVICE)
    edited = KERNEL.replace("// every row", "// every row of the tile\n\n").replace("/* one add */", "")
    assert bench.kernel_source_sha("pull", edited, "\n" + DEVICE + "// more\n") == base


def test_source_hash_follows_code_changes():
    base = bench.kernel_source_sha("pull", KERNEL, DEVICE)
    assert bench.kernel_source_sha("pull", KERNEL.replace("+= w[t]", "+= 2 * w[t]"), DEVICE) != base
    assert bench.kernel_source_sha("pull", KERNEL, DEVICE.replace("63", "31")) != base
    # a different kernel in the same file does not matter
    other = KERNEL + "template <typename T>\n__global__ void k_push(int t) {\n    t += 1;\n}\n"
    assert bench.kernel_source_sha("pull", other, DEVICE) == base


def test_source_hash_of_the_real_gather_kernel():
    sha = bench.kernel_source_sha("pull")
    assert len(sha) == 12 and int(sha, 16) >= 0


@pytest.fixture
def profiles_root(tmp_path, monkeypatch):
    """A copy of the package sources' location with a profiles/ folder of its own."""
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # kernel_source_sha reads the sources under ROOT: point it at the real ones
    src = os.path.join(ROOT, "paper_2302_03245_amd")
    os.symlink(src, tmp_path / "paper_2302_03245_amd")
    return tmp_path


def _record(root, tile, sha, alg, hbm):
    d = {"kernel": "k_pull", "tile_items": tile, "kernel_source_sha": sha,
         "algorithmic_bytes_per_launch": alg, "hbm_bytes_per_launch": hbm}
    (root / "profiles" / f"traffic_pull_wl_t{tile}.json").write_text(json.dumps(d))


def test_traffic_reported_for_matching_counters(profiles_root):
    sha = bench.kernel_source_sha("pull")
    _record(profiles_root, 2048, sha, 1.0e8, 1.2e8)
    assert bench.traffic_from_profiles("pull", "wl", 1.0e8, 2048) == 1.2e8
    assert bench.traffic_from_profiles("pull", "wl", 1.0e8 * 1.009, 2048) == 1.2e8  # within 1 %


def test_traffic_null_for_another_tile_size(profiles_root):
    _record(profiles_root, 2048, bench.kernel_source_sha("pull"), 1.0e8, 1.2e8)
    assert bench.traffic_from_profiles("pull", "wl", 1.0e8, 4096) is None


def test_traffic_null_for_other_launch_sizes(profiles_root):
    # a synchronous schedule (one gather per sweep) priced with an ordered one's counters
    _record(profiles_root, 2048, bench.kernel_source_sha("pull"), 1.0e8, 1.2e8)
    assert bench.traffic_from_profiles("pull", "wl", 3.3e8, 2048) is None


def test_traffic_null_after_a_kernel_change(profiles_root):
    _record(profiles_root, 2048, "0" * 12, 1.0e8, 1.2e8)
    assert bench.traffic_from_profiles("pull", "wl", 1.0e8, 2048) is None


def test_traffic_null_without_a_record(profiles_root):
    assert bench.traffic_from_profiles("pull", "other", 1.0e8, 2048) is None


def test_committed_traffic_records_are_well_formed():
    names = [f for f in os.listdir(os.path.join(ROOT, "profiles")) if f.startswith("traffic_")]
    assert names
    for f in names:
        d = json.load(open(os.path.join(ROOT, "profiles", f)))
        assert f.endswith(f"_t{d['tile_items']}.json"), f
        assert d["hbm_bytes_per_launch"] > 0 and d["algorithmic_bytes_per_launch"] > 0
        assert len(d["kernel_source_sha"]) == 12
        assert any("FETCH_SIZE" in c for c in d["commands"]) and any("WRITE_SIZE" in c for c in d["commands"])
