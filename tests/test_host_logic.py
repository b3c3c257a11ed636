"""Host-side logic that needs no GPU: the stats structure shared by the C header and the ctypes
binding, the benchmark's refusal of more than one GPU, and its rule for reporting HBM traffic only
from counters taken on the current panel source."""
import hashlib
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

C_TO_CTYPES = {"double": "c_double", "int64_t": "c_int64", "int32_t": "c_int32"}


def header_stats_fields():
    text = open(os.path.join(ROOT, "include", "rpca.h")).read()
    end = text.index("} rpca_stats;")
    body = text[text.rindex("typedef struct {", 0, end) + len("typedef struct {"):end]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    return re.findall(r"^\s*(double|int64_t|int32_t)\s+(\w+)\s*;", body, flags=re.M)


def test_stats_struct_matches_header():
    import ctypes
    from paper_1007_5510_amd import _lib
    fields = header_stats_fields()
    py = [(name, ctype) for name, ctype in _lib.Stats._fields_]
    assert [n for _, n in fields] == [n for n, _ in py]
    for (ctype_c, name), (_, ctype_py) in zip(fields, py):
        assert getattr(ctypes, C_TO_CTYPES[ctype_c]) is ctype_py, name


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_reported_only_for_the_profiled_source(tmp_path, monkeypatch):
    import bench
    src_dir = tmp_path / "paper_1007_5510_amd" / "csrc"
    src_dir.mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    src = src_dir / "panel_f32.hip"
    src.write_text("// kernel source\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()[:16]
    (tmp_path / "profiles" / "incore_f32_hbm_counters.md").write_text(
        f"traffic fwd32_kernel {sha} 1000 200\ntraffic adj_f32_kernel 0000000000000000 5 5\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("fwd32_kernel") == {"fetch": 1000.0, "write": 200.0}
    assert bench.measured_traffic("adj_f32_kernel") is None  # counters of another source
    src.write_text("// kernel source, changed\n")
    assert bench.measured_traffic("fwd32_kernel") is None


def test_traffic_of_another_source_uses_its_own_summary(tmp_path, monkeypatch):
    import bench
    src_dir = tmp_path / "paper_1007_5510_amd" / "csrc"
    src_dir.mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    (src_dir / "panel_f32.hip").write_text("// float32 kernels\n")
    x6 = src_dir / "panel_x6.hip"
    x6.write_text("// split kernels\n")
    sha = hashlib.sha256(x6.read_bytes()).hexdigest()[:16]
    (tmp_path / "profiles" / "incore_split_hbm_counters.md").write_text(f"traffic fwd_x6_kernel {sha} 300 40\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("fwd_x6_kernel", "panel_x6.hip", "incore_split_hbm_counters.md") == \
        {"fetch": 300.0, "write": 40.0}
    assert bench.measured_traffic("fwd_x6_kernel") is None  # not in the float32 summary
