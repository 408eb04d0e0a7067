"""Host logic of bench.py: the roofline object of the dominant kernel slot and
the committed traffic records it reads (no GPU)."""
import bench


def _slot(ms, launches, nbytes, flops):
    return dict(ms=ms, launches=launches, bytes=nbytes, flops=flops)


def test_roofline_picks_slot_with_most_device_time():
    kst = dict(gram=_slot(30.0, 10, 1.6e10, 1.5e12), admm32=_slot(20.0, 100, 2.0e10, 5e11),
               admm64=_slot(5.0, 10, 5e9, 1e11), plain=_slot(0.0, 0, 0.0, 0.0))
    r = bench.roofline(kst)
    assert r["slot"] == "gram" and r["launches"] == 10
    # 1.5e12 flop in 30 ms = 50 TFLOP/s against the float64 matrix peak; the
    # HBM time of 1.6e10 bytes (2 ms at 8 TB/s) is below the MFMA time (19 ms)
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s"
    assert abs(r["achieved"] - 50.0) < 1e-9
    assert abs(r["frac"] - round(50.0 / bench.PEAK_TFLOPS["f64"], 4)) < 1e-12
    assert r["avg_launch_us"] == 3000.0
    assert r["algorithmic_flops_per_launch"] == 150_000_000_000


def test_roofline_hbm_bound_slot():
    # 2e10 bytes and 1e11 flop in 10 ms: 2000 GB/s; HBM time 2.5 ms > MFMA time
    kst = dict(admm32=_slot(10.0, 4, 2.0e10, 1e11), gram=_slot(1.0, 1, 1.0, 1.0))
    r = bench.roofline(kst, "no_such_workload")
    assert r["slot"] == "admm32" and r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert abs(r["achieved"] - 2000.0) < 1e-9
    assert abs(r["frac"] - 0.25) < 1e-12
    assert r["traffic"] is None  # no counter record for that workload


def test_stored_traffic_follows_the_sources(tmp_path, monkeypatch):
    """A committed counter record counts only while the kernel's sources hash to
    the digest it was taken on."""
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "traffic_gram_w.txt").write_text("# header\nsources_sha256: abc123\ntraffic_bytes_per_launch: 4096\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "sources_digest", lambda files: "abc123")
    assert bench.stored_traffic("gram", "w") == 4096.0
    monkeypatch.setattr(bench, "sources_digest", lambda files: "changed")
    assert bench.stored_traffic("gram", "w") is None
    assert bench.stored_traffic("gram", "no_such_workload") is None


def test_committed_records_are_current_or_void():
    # the committed records either match their sources or are reported as null
    for slot in ("gram", "admm32"):
        t = bench.stored_traffic(slot)
        assert t is None or t > 1e8
