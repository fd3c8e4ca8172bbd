"""Host logic of bench.py, without a GPU: the kernel-source hash ignores
comments and blank lines but not code (so recorded counters stay valid
across comment edits only), and the traffic figure is the record of the
same sources and tile shape."""
import bench


def _reader(texts):
    return lambda rel: texts[rel]


def _sources():
    import os
    return {rel: open(os.path.join(bench.ROOT, rel), encoding="utf-8").read() for rel in bench.KERNEL_SOURCES}


def test_code_only_strips_comments_not_strings():
    src = 'int a = 1; // note\n/* block\n comment */ const char *s = "x // y /* z */";\n\n  int b;  \n'
    out = bench._code_only(src)
    assert "note" not in out and "block" not in out
    assert '"x // y /* z */"' in out
    assert out.splitlines() == ["int a = 1;", ' const char *s = "x // y /* z */";', "  int b;"]


def test_hash_ignores_comments_but_not_code():
    texts = _sources()
    h0 = bench.kernel_source_hash(read=_reader(texts))
    assert h0 == bench.kernel_source_hash()
    rel = bench.KERNEL_SOURCES[0]
    commented = dict(texts)
    commented[rel] = texts[rel].replace("\n", "\n// an added comment\n", 1) + "\n/* trailing */\n\n"
    assert bench.kernel_source_hash(read=_reader(commented)) == h0
    changed = dict(texts)
    changed[rel] = texts[rel] + "\nconstexpr int EXTRA = 1;\n"
    assert bench.kernel_source_hash(read=_reader(changed)) != h0


def test_traffic_record_matches_sources_and_shape(monkeypatch):
    h = bench.kernel_source_hash()
    recs = [{"kernel_sources": "0" * 16, "schedule": [8, 1], "bytes_per_launch": 1.0},
            {"kernel_sources": h, "schedule": [4, 1], "bytes_per_launch": 2.0},
            {"kernel_sources": h, "schedule": [8, 1], "bytes_per_launch": 3.0}]
    monkeypatch.setattr(bench, "_traffic_records", lambda: recs)
    assert bench.measured_traffic({"wave_rows": 8, "waves_x": 1})["bytes_per_launch"] == 3.0
    assert bench.measured_traffic({"wave_rows": 4, "waves_x": 1})["bytes_per_launch"] == 2.0
    assert bench.measured_traffic({"wave_rows": 16, "waves_x": 1}) is None
    monkeypatch.setattr(bench, "_traffic_records", lambda: recs[:1])
    assert bench.measured_traffic({"wave_rows": 8, "waves_x": 1}) is None


def test_committed_summary_parses():
    recs = bench._traffic_records()
    assert recs, "the committed counter summary holds at least one record"
    for r in recs:
        assert r["bytes_per_launch"] == r["fetch_bytes"] + r["write_bytes"]
        assert len(r["schedule"]) == 2 and len(r["kernel_sources"]) == 16


def test_profile_names_are_the_librarys():
    """The benchmark drains every per-launch timing name the library keeps,
    so that its timed sections leave no events behind."""
    import re
    src = _sources()["paper_2211_16266_amd/csrc/pms.hip"]
    block = re.search(r"kKernelNames\[kNumKernelKinds\]\s*=\s*\{(.*?)\};", src, re.S).group(1)
    names = tuple(re.findall(r'"([a-z_]+)"', block))
    assert names == bench.PROFILE_NAMES
    assert set(bench.NEXT_BYTES) <= set(names)


def test_util_summary_means_and_derived_figures(tmp_path):
    """Per-dispatch means over the named kernel's dispatches (rows of one
    dispatch and counter summed), GRBM_GUI_ACTIVE taken from the first pass,
    and the derived utilisation figures from them."""
    import csv
    head = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]

    def write(d, rows):
        d.mkdir()
        with open(d / "pmc_counter_collection.csv", "w", newline="") as f:
            w = csv.writer(f)
            w.writerow(head)
            w.writerows(rows)

    k, other = "void pms::k_tiles<1, 0, 4, 9, true>(pms::Launch)", "pms::k_pad(pms::Launch)"
    cyc = 1000.0
    write(tmp_path / "a", [
        [1, k, "GRBM_GUI_ACTIVE", 8 * cyc], [1, k, "SQ_INSTS_VALU", 0.5 * 1024 * cyc / 4],
        [1, k, "SQ_INSTS_VMEM_RD", 10.0], [1, k, "SQ_WAVES", 5.0],
        [1, k, "TCP_TOTAL_CACHE_ACCESSES_sum", 150.0], [1, k, "TCP_TOTAL_CACHE_ACCESSES_sum", 150.0],
        [2, k, "GRBM_GUI_ACTIVE", 8 * cyc], [2, k, "SQ_INSTS_VALU", 0.7 * 1024 * cyc / 4],
        [2, k, "SQ_INSTS_VMEM_RD", 10.0], [2, k, "SQ_WAVES", 5.0],
        [2, k, "TCP_TOTAL_CACHE_ACCESSES_sum", 300.0],
        [3, other, "SQ_INSTS_VALU", 1e12],
    ])
    write(tmp_path / "b", [
        [1, k, "GRBM_GUI_ACTIVE", 99.0], [1, k, "SQ_LDS_IDX_ACTIVE", 0.1 * 256 * cyc],
        [1, k, "SQ_LDS_BANK_CONFLICT", 0.02 * 256 * cyc],
    ])
    out = bench.util_summary("k_tiles<1, 0, 4, 9, true>", [str(tmp_path / "a"), str(tmp_path / "b")])
    lines = {ln.split("|")[1].strip(): ln.split("|")[2].strip() for ln in out.splitlines() if ln.startswith("| ")}
    assert float(lines["GRBM_GUI_ACTIVE"]) == 8 * cyc
    assert lines["VALU issue: SQ_INSTS_VALU x 4 / (1024 SIMDs x cycles)"] == "0.600"
    assert lines["L1 lookups per vector load: TCP_TOTAL_CACHE_ACCESSES_sum / SQ_INSTS_VMEM_RD"] == "30.0"
    assert lines["LDS indexed-access busy: SQ_LDS_IDX_ACTIVE / (256 x cycles)"] == "0.1000"
    assert lines["LDS conflict cycles per conflict-free LDS cycle: SQ_LDS_BANK_CONFLICT / "
                 "(SQ_LDS_IDX_ACTIVE - SQ_LDS_BANK_CONFLICT)"] == "0.2500"
