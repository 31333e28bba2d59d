"""bench.py's reading of the committed rocprofv3 counter summaries: HBM bytes
per launch are taken only while the kernel code they were measured on is
unchanged (comments aside) and only for the launch shape recorded."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _write(tmp_path, digest, entries):
    p = tmp_path / "summary.md"
    lines = ["# a summary", "", "Machine-readable:", "", f"    source_digest: {digest}  (note)"]
    lines += [f"    shape {k}: traffic_bytes_per_launch {v} kernel_avg_us 1.0" for k, v in entries.items()]
    p.write_text("\n".join(lines) + "\n")
    return str(p)


def test_digest_ignores_comments_not_code(tmp_path):
    a = tmp_path / "a.hpp"
    b = tmp_path / "b.hpp"
    a.write_text("int f() {\n  return 1;  // one\n}\n/* block */\n")
    b.write_text("// header\nint f() {\n  return 1;\n}\n\n")
    assert bench.kernel_source_digest(str(a)) == bench.kernel_source_digest(str(b))
    b.write_text("int f() {\n  return 2;\n}\n")
    assert bench.kernel_source_digest(str(a)) != bench.kernel_source_digest(str(b))
    # several sources are read in order
    assert bench.kernel_source_digest((str(a), str(b))) != bench.kernel_source_digest((str(b), str(a)))


def test_traffic_only_for_current_code_and_recorded_shape(tmp_path):
    src = tmp_path / "k.hpp"
    src.write_text("int k;\n")
    path = _write(tmp_path, bench.kernel_source_digest(str(src)), {"1,112": 697253080, "born,336": 12345})
    assert bench.profiled_traffic((1, 112), path, str(src)) == 697253080.0
    assert bench.profiled_traffic(("born", 336), path, str(src)) == 12345.0
    assert bench.profiled_traffic((3, 56), path, str(src)) is None          # shape not profiled
    src.write_text("int k2;\n")                                               # the kernel changed
    assert bench.profiled_traffic((1, 112), path, str(src)) is None
    assert bench.profiled_traffic((1, 112), str(tmp_path / "missing.md"), str(src)) is None


@pytest.mark.parametrize("name,src,shape", [
    ("step3d_o8_336cube_forward.md", bench.KERNEL_SRC, (1, 112)),
    ("step3d_o16_480cube_forward.md", bench.KERNEL_SRC, (3, 240)),
    ("step3d_o16_480cube_gradient_imaging.md", bench.KERNEL_SRC, (2, 240)),
    ("born3d_o8_336cube_born.md", bench.BORN_SRC, ("born", 336)),
])
def test_committed_summaries_parse(name, src, shape):
    path = os.path.join(ROOT, "profiles", name)
    v = bench.profiled_traffic(shape, path, src)
    # None only when the kernel code has moved on since the counters were taken
    assert v is None or v > 0
