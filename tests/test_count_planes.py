"""The kernels' bit-sliced count helpers checked exhaustively on the host (CPU).

The tile routine keeps every row's count in bit planes (the bit-sliced index of
Section 5.3.1) and compares them with the threshold plane by plane, reads the largest
count for opt-threshold queries, and reads single rows' counts back for the histogram
and general symmetric tables.  These helpers are __host__ __device__ functions of the
kernel header; tests/csrc/count_planes_check.cpp includes that header, builds for the
host only and checks them against integer arithmetic for every count 0..N' and every
threshold, N' <= 1024.  The layout helpers of the fine presence records are checked the same
way (tests/csrc/record_layout_check.cpp), and so is the bounds pre-pass's item order
(tests/csrc/pre_order_check.cpp).
"""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_bit_sliced_helpers_exhaustive(tmp_path):
    exe = str(tmp_path / "count_planes_check")
    subprocess.run([HIPCC, "-x", "hip", "--offload-host-only", "-O2", "-std=c++17",
                    "-I", os.path.join(ROOT, "paper_1402_4466_amd", "csrc"), "-o", exe,
                    os.path.join(ROOT, "tests", "csrc", "count_planes_check.cpp")],
                   check=True, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.startswith("ok"), r.stdout


def test_presence_record_layout(tmp_path):
    """The fine presence records' four arrays (per-word, quarter and two 8-row halves) are
    disjoint, in order, on 128-byte lines per tile and within 32-bit word offsets for every
    tile count a registered bitmap can have (tests/csrc/record_layout_check.cpp)."""
    exe = str(tmp_path / "record_layout_check")
    subprocess.run([HIPCC, "-x", "hip", "--offload-host-only", "-O2", "-std=c++17",
                    "-I", os.path.join(ROOT, "paper_1402_4466_amd", "csrc"), "-o", exe,
                    os.path.join(ROOT, "tests", "csrc", "record_layout_check.cpp")],
                   check=True, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.startswith("ok"), r.stdout


def test_prepass_item_order(tmp_path):
    """The bounds pre-pass's item order maps every XCD share of a batch onto itself one to one and
    takes a share of whole queries in blocks of tiles across its queries, for every batch of up to
    72 queries of up to 70 tiles, larger batches and workgroups of 1 to 16 wavefronts
    (tests/csrc/pre_order_check.cpp)."""
    exe = str(tmp_path / "pre_order_check")
    subprocess.run([HIPCC, "-x", "hip", "--offload-host-only", "-O2", "-std=c++17",
                    "-I", os.path.join(ROOT, "paper_1402_4466_amd", "csrc"), "-o", exe,
                    os.path.join(ROOT, "tests", "csrc", "pre_order_check.cpp")],
                   check=True, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.startswith("ok"), r.stdout
