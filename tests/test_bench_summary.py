"""The counter summary behind bench.py's `traffic` field, on synthetic
rocprofv3 counter files (no GPU): each counter is scaled by the factor that
makes the 256 MiB calibration copies read 256 MiB (small copies are left out
of that factor), and a kernel's mean per launch leaves out the dispatches that
did no work (launches the device skipped)."""
import csv
import os

import bench

HEADER = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
KERNEL = "void fnls::k_pass<double, 4, 10, 0, 16, 0, 2, 1>(fnls::PassArgs)"


def write_run(path, counter, copies, small_copy, kernel_vals):
    os.makedirs(path, exist_ok=True)
    rows = []
    for v in copies:
        rows.append([len(rows), bench.COPY_KERNEL, counter, v])
    rows.append([len(rows), bench.COPY_KERNEL, counter, small_copy])
    for v in kernel_vals:
        rows.append([len(rows), KERNEL, counter, v])
    with open(os.path.join(path, "x_counter_collection.csv"), "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(HEADER)
        w.writerows(rows)


def keyvals(text):
    out = {}
    for line in text.splitlines():
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            out[k] = v
    return out


def test_traffic_scales_by_the_copies_and_skips_idle_dispatches(tmp_path, capsys):
    mib = 1024.0   # KiB per MiB
    # the copies read 256 MiB as 230.4 MiB (FETCH) and 460.8 MiB (WRITE)
    write_run(str(tmp_path / "f"), "FETCH_SIZE", [230.4 * mib] * 3, 6.5, [0.0, 90.0 * mib, 110.0 * mib, 0.2])
    write_run(str(tmp_path / "w"), "WRITE_SIZE", [460.8 * mib] * 3, 3.0, [40.0 * mib, 0.0, 40.0 * mib])
    bench.summarize([str(tmp_path / "f"), str(tmp_path / "w")], "pass64.toep_next_wdots.ax0",
                    r"k_pass<double, 4, 10, 0, 16, 0, 2, 1>")
    kv = keyvals(capsys.readouterr().out)
    f_fac, w_fac = 256.0 / 230.4, 256.0 / 460.8
    assert abs(float(kv["fetch_size_copy_factor"]) - f_fac) < 1e-4
    assert abs(float(kv["write_size_copy_factor"]) - w_fac) < 1e-4
    # mean of the two working dispatches (100 MiB), not of all four
    fetch = 100.0 * (1 << 20) * f_fac
    write = 40.0 * (1 << 20) * w_fac
    assert abs(float(kv["fetch_size_bytes_per_launch"]) - fetch) < 2.0
    assert abs(float(kv["write_size_bytes_per_launch"]) - write) < 2.0
    assert abs(float(kv["hbm_bytes_per_launch"]) - (fetch + write)) < 2.0
    assert kv["source_sha256"] == bench.source_hash()
