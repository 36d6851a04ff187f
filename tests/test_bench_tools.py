"""The benchmark's profile summarisers on synthetic rocprofv3 CSV files (no
GPU): kernel names with parameter lists and anonymous namespaces, the copy
calibration, the sum of a kernel's instances per call, probes left out."""
import csv
import os

import pytest

import bench

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def write_csv(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(FIELDS, r)))


def test_kernel_name():
    assert bench.kernel_name("void hc::k_encode<true, 2u, 4u>(hc::JobList, unsigned int)") == \
        "hc::k_encode<true, 2u, 4u>"
    assert bench.kernel_name("(anonymous namespace)::k_probe_copy(unsigned int __vector(4) const*, unsigned long)") == \
        "k_probe_copy"
    assert bench.kernel_name("hc::k_hist(hc::JobList, unsigned long)") == "hc::k_hist"


def test_traffic_summary(tmp_path):
    gib = 1 << 30
    ring = "void hc::k_decode_ring<16u, 3u, false, false>(hc::JobList, unsigned int)"
    copy = "void hc::k_decode_ring<16u, 4u, false, true>(hc::JobList, unsigned int)"
    probe_c = "(anonymous namespace)::k_probe_copy(unsigned int __vector(4) const*, unsigned int __vector(4)*)"
    probe_r = "(anonymous namespace)::k_probe_read(unsigned int __vector(4) const*, unsigned long)"
    kib = lambda nbytes: nbytes / 1024.0
    root = str(tmp_path / "pmc")
    # FETCH_SIZE reads half the bytes a copy fetches, WRITE_SIZE all it writes
    write_csv(f"{root}/fetch/run_counter_collection.csv",
              [(1, ring, "FETCH_SIZE", kib(3 << 29)), (2, ring, "FETCH_SIZE", kib(3 << 29)),
               (3, copy, "FETCH_SIZE", kib(1 << 29)), (4, probe_c, "FETCH_SIZE", kib(gib // 2))])
    write_csv(f"{root}/write/run_counter_collection.csv",
              [(1, ring, "WRITE_SIZE", kib(2 * gib)), (3, copy, "WRITE_SIZE", kib(gib))])
    write_csv(f"{root}/copy_fetch/run_counter_collection.csv",
              [(1, probe_c, "FETCH_SIZE", kib(gib // 2)), (2, probe_r, "FETCH_SIZE", kib(gib // 2))])
    write_csv(f"{root}/copy_write/run_counter_collection.csv",
              [(1, probe_c, "WRITE_SIZE", kib(gib)), (2, probe_r, "WRITE_SIZE", kib(1 << 10))])
    out = bench.traffic_summary(root, 65536, 1024, out_dir=str(tmp_path))
    assert set(out) == {"k_decode_ring"}  # the probes are not codec kernels
    rec = out["k_decode_ring"]
    assert rec["copy_kernel"] == "k_probe_copy"
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    # both instances, once each per call: FETCH (1.5 + 0.5) GiB x 2 read, WRITE (2 + 1) GiB written
    assert rec["bytes_per_launch"] == pytest.approx(4 * gib + 3 * gib, rel=1e-6)
    assert os.path.exists(tmp_path / "traffic_k_decode_ring_mixed-4GiB-64x64MiB_B65536_S1024.json")


def test_sq_table_takes_each_kinds_timed_dispatch(tmp_path, capsys):
    class Args:
        segments, steps, warmup = 4, 1, 1

    import synth

    symbols = 4 * synth.WORKLOADS[bench.WORKLOAD]["segment"]
    names = ["void hc::k_count<4u>(x)", "void hc::k_encode<true, 2u, 4u>(x)",
             "void hc::k_decode_ring<16u, 3u, false, false>(x)"]
    rows, d = [], 0
    for kind in range(3):
        for rep in range(2):  # warm-up pass, then the timed pass
            for k, n in enumerate(names):
                d += 1
                valu = (symbols // 64) * (100 * kind + 10 * k + rep + 1)  # rep 1: the timed pass
                for c, v in (("SQ_INSTS_VALU", valu), ("SQ_INSTS_LDS", 0), ("SQ_WAVE_CYCLES", 1000),
                             ("SQ_WAIT_ANY", 250), ("SQ_WAIT_INST_ANY", 250), ("SQ_ACTIVE_INST_ANY", 500),
                             ("SQ_LDS_BANK_CONFLICT", 0), ("SQ_ACTIVE_INST_LDS", 1)):
                    rows.append((d, n, c, v))
    write_csv(str(tmp_path / "sq" / "run_counter_collection.csv"), rows)
    bench.sq_table(str(tmp_path), synth, Args())
    out = [l for l in capsys.readouterr().out.splitlines() if l.startswith("| ") and "kernel" not in l]
    assert len(out) == 9
    # fp32 (kind 2), packing pass (k = 1), timed pass: 100*2 + 10*1 + 2 VALU per symbol
    fp32_pack = next(l for l in out if l.startswith("| fp32 | `k_encode"))
    assert fp32_pack.split("|")[3].strip() == "212.00"
    assert fp32_pack.split("|")[6].strip() == "0.25" and fp32_pack.split("|")[8].strip() == "0.50"
