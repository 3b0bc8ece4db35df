"""bench.py pieces that run without a GPU: the one-GPU guard, the oracle
baseline leg, and the counter summary / traffic record round trip."""
import csv
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import oracle  # noqa: E402
from paper_2006_08861_amd import workload  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_cpu_baseline_times_the_oracle():
    w = workload.make_workload(0, nq=6)
    ref = oracle.retrieve(w.feats, w.region_of, w.n_regions_total, w.q, w.k, w.n_reg)
    base, recall, exact, m = bench.cpu_baseline(w, np.asarray(ref["idx"]), 0.2)
    assert base["kind"] == "oracle" and base["value"] > 0 and base["single_core_value"] > 0
    assert base["cores"] == bench.oracle_threads() and 1 <= base["cores"] <= 16
    assert recall == 1.0 and exact == m and m == len(w.q)


def test_cpu_baseline_samples_whole_requests():
    # above the full-batch size the oracle is timed on the first whole
    # requests holding at least the sample size
    w = workload.make_workload(3, nq=40, n=20_000)
    ref = oracle.retrieve(w.feats, w.region_of, w.n_regions_total, w.q, w.k, w.n_reg)
    base, recall, exact, m = bench.cpu_baseline(w, np.asarray(ref["idx"]), 0.2,
                                                sample_frames=20, full_rows=1000)
    assert m == 24 and "first 3 requests" in base["sample"]
    assert recall == 1.0 and exact == m


def _csv(path, rows):
    with open(path, "w", newline="") as f:
        wr = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name",
                                           "Counter_Value"])
        wr.writeheader()
        for r in rows:
            wr.writerow(r)


def test_counter_summary_round_trip(tmp_path, monkeypatch, capsys):
    # one record per rows-per-item tile; the dense (coarse) dispatches of the
    # same template are not counted
    narrow = "void hloc::k_screen_blk<16, false, false>(hloc::ScreenArgs)"
    hoist = "void hloc::k_screen_blk<16, true, false>(hloc::ScreenArgs)"
    dense = "void hloc::k_screen_blk<16, false, true>(hloc::ScreenArgs)"
    wide = "void hloc::k_screen_wide<16>(hloc::ScreenArgs)"
    copy = ("void at::native::vectorized_elementwise_kernel<4, at::native::CUDAFunctorOnSelf_add"
            "<float>, std::array<char*, 2ul> >(int)")
    # per step: the coarse stage (dense narrow kernel, or the wide kernel in
    # dense mode for large batches), then the fine narrow and wide launches;
    # only the wide launch that follows a narrow list launch is the fine one
    steps = [(dense, 9000, 900), (wide, 7777, 777), (narrow, 100, 8), (wide, 10, 2),
             (dense, 9000, 900), (wide, 7777, 777), (narrow, 300, 8), (wide, 10, 2)]
    _csv(tmp_path / "f.csv", [dict(Dispatch_Id=j + 1, Kernel_Name=k, Counter_Name="FETCH_SIZE",
                                   Counter_Value=fv) for j, (k, fv, _) in enumerate(steps)])
    _csv(tmp_path / "w.csv", [dict(Dispatch_Id=j + 1, Kernel_Name=k, Counter_Name="WRITE_SIZE",
                                   Counter_Value=wv) for j, (k, _, wv) in enumerate(steps)])
    _csv(tmp_path / "f2.csv", [dict(Kernel_Name=hoist, Counter_Name="FETCH_SIZE", Counter_Value=150),
                               dict(Kernel_Name=wide, Counter_Name="FETCH_SIZE", Counter_Value=10)])
    _csv(tmp_path / "w2.csv", [dict(Kernel_Name=hoist, Counter_Name="WRITE_SIZE", Counter_Value=6),
                               dict(Kernel_Name=wide, Counter_Name="WRITE_SIZE", Counter_Value=2)])
    _csv(tmp_path / "cf.csv", [dict(Kernel_Name=copy, Counter_Name="FETCH_SIZE", Counter_Value=512)])
    _csv(tmp_path / "cw.csv", [dict(Kernel_Name=copy, Counter_Name="WRITE_SIZE", Counter_Value=1024)])

    class A:
        counters_summary = [str(tmp_path / n) for n in ("f.csv", "w.csv", "cf.csv", "cw.csv")]
        precision = "fp32"
        copy_mib = 1
        workload_name = "unit"
        commands = ["cmd"]
        tiles = "64,16"
        counters_append = False

    bench.counters_summary(A)
    A.counters_summary = [str(tmp_path / n) for n in ("f2.csv", "w2.csv", "cf.csv", "cw.csv")]
    A.tiles, A.counters_append = "128,4", True
    bench.counters_summary(A)
    text = capsys.readouterr().out
    recs = [json.loads(line[len("record: "):]) for line in text.splitlines()
            if line.startswith("record: ")]
    assert [r["rows_per_item"] for r in recs] == [64, 128]
    assert "k_screen_blk<NS, true, false>" in recs[1]["kernel"]
    # narrow mean 200 KiB + wide 10 KiB fetched, scaled by 1 MiB / 512 KiB = 2
    assert recs[0]["fetch_kib"] == 210.0 and recs[0]["fetch_scale"] == 2.0
    assert recs[0]["write_kib"] == 10.0 and recs[0]["write_scale"] == 1.0
    assert recs[1]["fetch_kib"] == 160.0 and recs[1]["write_kib"] == 8.0
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "counters_screen_fp32_unit.md").write_text(text)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "screen_digest", lambda: recs[0]["sources"])
    b, src = bench.load_traffic("unit", "fp32", 64)
    assert b == 1024.0 * (210.0 * 2.0 + 10.0 * 1.0)
    b, src = bench.load_traffic("unit", "fp32", 128)
    assert b == 1024.0 * (160.0 * 2.0 + 8.0 * 1.0)
    b, src = bench.load_traffic("unit", "fp32", 32)
    assert b is None and "32-row" in src
    monkeypatch.setattr(bench, "screen_digest", lambda: "changed")
    b, src = bench.load_traffic("unit", "fp32", 64)
    assert b is None and "changed" in src


def test_fft_counter_record_round_trip(tmp_path, monkeypatch, capsys):
    """The feature kernel's summary: per-dispatch FETCH/WRITE scaled by the
    copy calibration, read back while the kernel source is unchanged."""
    name = bench.fft_workload_name(200_000, 512, 256)
    assert name == "fft-200k-L512-d256"
    kname = bench.fft_kernel_name(512)
    assert kname == "k_fft_magnitude_sq<16>" and bench.fft_kernel_name(1024) == "k_fft_magnitude"
    full = f"void hloc::{kname}(float const*, long, int, float*)"
    copy = "void at::native::vectorized_elementwise_kernel<4, at::native::CUDAFunctorOnSelf_add<float> >"
    f_csv, w_csv = str(tmp_path / "f.csv"), str(tmp_path / "w.csv")
    cf_csv, cw_csv = str(tmp_path / "cf.csv"), str(tmp_path / "cw.csv")
    _csv(f_csv, [dict(Dispatch_Id=i, Kernel_Name=full, Counter_Name="FETCH_SIZE",
                      Counter_Value=300_000.0) for i in range(3)])
    _csv(w_csv, [dict(Dispatch_Id=i, Kernel_Name=full, Counter_Name="WRITE_SIZE",
                      Counter_Value=200_000.0) for i in range(3)])
    _csv(cf_csv, [dict(Dispatch_Id=0, Kernel_Name=copy, Counter_Name="FETCH_SIZE",
                       Counter_Value=512.0)])
    _csv(cw_csv, [dict(Dispatch_Id=0, Kernel_Name=copy, Counter_Name="WRITE_SIZE",
                       Counter_Value=1024.0)])

    class A:
        fft_counters = (f_csv, w_csv, cf_csv, cw_csv)
        fft_signals, fft_len, fft_bins, copy_mib = 200_000, 512, 256, 1
        commands = ["cmd"]

    bench.fft_counters_summary(A)
    text = capsys.readouterr().out
    assert "record: " in text
    monkeypatch.setattr(bench, "fft_counters_path", lambda n: str(tmp_path / "c.md"))
    (tmp_path / "c.md").write_text(text)
    traffic, src = bench.load_fft_traffic(name)
    assert traffic == 1024.0 * (300_000.0 * 2.0 + 200_000.0 * 1.0)
    monkeypatch.setattr(bench, "fft_digest", lambda: "another")
    traffic, src = bench.load_fft_traffic(name)
    assert traffic is None and "changed" in src


def test_committed_fft_record_matches_the_kernel_source():
    """The committed counters of the feature kernel: about the algorithmic
    bytes (each signal read once, each bin written once). After a change to
    the kernel the benchmark reports no traffic until they are taken again."""
    import pytest
    traffic, src = bench.load_fft_traffic("fft-200k-L512-d256")
    if traffic is None:
        pytest.skip(f"no current counter record: {src}")
    assert abs(traffic / (200_000 * 4 * (512 + 256)) - 1.0) < 0.01


def test_committed_screen_records_cover_the_tuner_tiles():
    """The committed fine-screen counters of the benchmark's default workload
    hold a record for every rows-per-item tile the tuner may choose, each
    between the algorithmic bytes of the batch (2.09 GB: every kept row's
    bf16 copy and norm, the frames, the block words) and twice that. After a
    change to the screen sources the benchmark reports no traffic until they
    are taken again."""
    import pytest
    algorithmic = 2.0896e9
    for rows in (32, 64, 96, 128):
        traffic, src = bench.load_traffic("fp8-2m-d512-8frame", "bf16", rows)
        if traffic is None and "changed" in src:
            pytest.skip(f"no current counter record: {src}")
        assert traffic is not None, (rows, src)
        assert algorithmic <= traffic <= 2.0 * algorithmic, (rows, traffic)
