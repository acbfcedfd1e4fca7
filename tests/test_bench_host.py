"""Host logic of bench.py that runs without a GPU: which committed counter
summary the roofline reads, and that a summary counts only for the kernel
and the build of its sources it was taken on."""
import os

import bench


def test_summary_file_per_kernel_family():
    assert bench._summary_name("k_gemm_wide_w8<5>", "hbm_traffic") == \
        "k_gemm_wide_3x3x3_hbm_traffic.txt"
    assert bench._summary_name("k_gemm_blk<5,4,2>", "issue_counters") == \
        "k_gemm_blk_3x3x3_issue_counters.txt"


def test_recorded_figures_tied_to_kernel_and_sources():
    path = os.path.join(bench.ROOT, "profiles", "k_gemm_wide_3x3x3_hbm_traffic.txt")
    assert os.path.exists(path)
    f = bench._summary_fields("k_gemm_wide_3x3x3_hbm_traffic.txt")
    kname = f["kernel"]
    assert kname in ("k_gemm_wide<5>", "k_gemm_wide_w8<5>")
    sha = f["source_sha"]
    assert bench.recorded_traffic(kname, sha) == float(f["traffic_bytes_per_launch"])
    # another kernel, or another build of the kernel sources: no figure
    assert bench.recorded_traffic(kname.replace("<5>", "<10>"), sha) is None
    assert bench.recorded_traffic(kname, "0" * 16) is None
    assert bench.recorded_issue(kname, "0" * 16) == {"blocked_issue_counters": None}
    got = bench.recorded_issue(kname, sha)["blocked_issue_counters"]
    assert got is not None and got["mfma_per_wave_tile"] > 0


def test_committed_summaries_match_the_kernel_sources():
    """Every committed wide-kernel summary names the build it was taken on;
    they were taken together, on the current kernel sources."""
    names = ["k_gemm_wide_3x3x3_hbm_traffic.txt", "k_gemm_wide_3x3x3_issue_counters.txt",
             "k_gemm_wide_3x3x3_full_map_kernel_trace.txt",
             "k_gemm_wide_6x6_full_map_kernel_trace.txt"]
    shas = {bench._summary_fields(n)["source_sha"] for n in names}
    assert shas == {bench.kernel_source_hash()}
    kernels = {bench._summary_fields(n)["kernel"] for n in names[:3]}
    assert kernels == {"k_gemm_wide_w8<5>"}
