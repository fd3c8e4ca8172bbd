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
