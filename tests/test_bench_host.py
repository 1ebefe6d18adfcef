"""Host-side pieces of bench.py: profiler-name parsing, the per-launch grouping of
counter rows, and the refusal of a summary taken on another kernel source."""
import os

import bench


def test_short_names_and_matching():
    n = "void fc::(anonymous namespace)::wilson_lds_kernel<false, true>(fc::CoopArgs, unsigned int)"
    assert bench._short(n) == "wilson_lds_kernel<false, true>"
    assert bench._short("fc::(anonymous namespace)::validate_rows_kernel(int const*, int)") == \
        "validate_rows_kernel"
    assert bench._matches(n, ["wilson_lds_kernel"])
    assert not bench._matches(n, ["wilson_lds"])
    assert not bench._matches("fc::lds_predraw_kernel<false>(x)", ["wilson_lds_kernel"])
    # another library's kernel of the same short name is not ours
    assert not bench._matches("void at::native::reduce_kernel<128, 4>(x)", ["reduce_kernel"])
    assert bench._matches("fc::(anonymous namespace)::reduce_kernel(double*)", ["reduce_kernel"])


def test_dispatch_counters_sum_per_dispatch():
    rows = []
    for d, name, vals in ((1, "fc::a_kernel(int)", {"TCC_HIT_sum": 3, "TCC_MISS_sum": 4}),
                          (2, "fc::other_kernel(int)", {"TCC_HIT_sum": 100, "TCC_MISS_sum": 1}),
                          (3, "void fc::b_kernel<1>(int)", {"TCC_HIT_sum": 5, "TCC_MISS_sum": 6})):
        for c, v in vals.items():
            rows.append({"Dispatch_Id": str(d), "Kernel_Name": name, "Counter_Name": c,
                         "Counter_Value": str(v)})
    got = bench._dispatch_counters(rows, ["a_kernel", "b_kernel"])
    assert sorted(got) == [1, 3]
    assert got[1] == ("a_kernel", {"TCC_HIT_sum": 3.0, "TCC_MISS_sum": 4.0})
    assert got[3][0] == "b_kernel<1>"


def test_summary_refused_on_another_source(tmp_path, monkeypatch):
    stem = "wilson_tile_grid1000"
    h = bench.kernel_hash(bench.PROFILE_SPECS[stem]["sources"])
    monkeypatch.setattr(bench, "PROFILE_DIR", str(tmp_path))
    p = tmp_path / f"{stem}_traffic.txt"
    p.write_text(f"# c\nkernel_source_sha256_16: {h}\nhbm_bytes_per_launch.alpha1.0: 1234\n")
    assert bench.traffic_of(stem, "alpha1.0") == 1234.0
    assert bench.traffic_of(stem, "alpha2.0") is None
    p.write_text("kernel_source_sha256_16: 0000000000000000\nhbm_bytes_per_launch.alpha1.0: 1\n")
    assert bench.traffic_of(stem, "alpha1.0") is None


def test_hash_covers_included_headers():
    files = bench.hashed_files(["wilson_tile.hip"])
    assert "wilson_tile.hip" in files and "fc_kernels.hpp" in files
    for f in files:
        assert os.path.exists(bench._src_path(f))


def test_roofline_fields():
    r = bench.roofline_hbm(8e9, 2.0, traffic=12e9)
    assert abs(r["achieved"] - 4000.0) < 1e-9 and abs(r["frac"] - 0.5) < 1e-12
    assert abs(r["traffic_frac"] - 0.75) < 1e-12
    assert abs(r["traffic_over_algorithmic"] - 1.5) < 1e-12
    assert bench.roofline_hbm(1.0, 1.0)["traffic"] is None


def test_host_info_share():
    h = bench.host_info()
    assert 1 <= h["cores_used"] <= h["affinity_cpus"] <= h["nproc"]


def test_line_ceiling_added_to_nested_rooflines():
    extras = {"grid": {"per_alpha": {"1.0": {"roofline": {"traffic": 6.6e9, "kernel_ms": 1.0}}}},
              "batch": {"batched": {"roofline": {"traffic": None, "kernel_ms": 2.0}}}}
    bench._add_line_ceiling(extras, 6.6e12)
    assert abs(extras["grid"]["per_alpha"]["1.0"]["roofline"]["random_line_ceiling_frac"] - 1.0) < 1e-12
    assert "random_line_ceiling_frac" not in extras["batch"]["batched"]["roofline"]


def test_code_tokens_ignore_comments_and_layout():
    a = "int f(int x) {  // add one\n    return x + 1; /* done */ }\n"
    b = "int f(int x)\n{\n    return x + 1;\n}\n"
    assert bench.code_tokens(a) == bench.code_tokens(b)
    assert bench.code_tokens('const char *s = "a // b";') == 'const char *s = "a // b";'
    assert bench.code_tokens("x = 1; // c") != bench.code_tokens("x = 2; // c")
