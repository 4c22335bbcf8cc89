"""Host-side parts of bench.py (no GPU): the one-GPU rule and the kernel-source digest that keys the
recorded HBM-traffic counters."""
import os
import shutil
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

CSRC = ("paper_1412_1840_amd", "csrc")


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and p.stdout == ""


def _copy_sources(tmp_path):
    dst = tmp_path.joinpath(*CSRC)
    dst.mkdir(parents=True)
    for name in ("qmi_kernels.hip", "qmi_internal.h"):
        shutil.copy(os.path.join(ROOT, *CSRC, name), dst / name)
    return dst


def test_digest_ignores_comments_and_white_space_only(tmp_path):
    base = bench.kernel_code_digest(ROOT)
    dst = _copy_sources(tmp_path)
    assert bench.kernel_code_digest(str(tmp_path)) == base
    k = dst / "qmi_kernels.hip"
    text = k.read_text()
    k.write_text("// an added comment\n/* and a block\n   comment */\n" + text.replace("\n", "\n\n"))
    assert bench.kernel_code_digest(str(tmp_path)) == base
    assert "constexpr int kRowFold = 64;" in text
    k.write_text(text.replace("constexpr int kRowFold = 64;", "constexpr int kRowFold = 128;"))
    assert bench.kernel_code_digest(str(tmp_path)) != base
