"""Host-side checks of the rocprofv3 summaries bench.py writes into profiles/
(no GPU needed): on small SQLite databases laid out like rocprofv3's result
databases, the kernel-trace summary groups launches per kernel and grid size
and reports allocated VGPRs, and the counter summary calibrates FETCH_SIZE
and WRITE_SIZE on the copy kernels of known size."""

import sqlite3

import pytest

import bench


def _trace_db(path, launches):
    con = sqlite3.connect(path)
    con.execute("create table kernel_symbols (kernel_id integer, kernel_name text)")
    con.execute("create table kernels (name text, kernel_id integer, grid_x integer, workgroup_x integer, "
                "vgpr_count integer, duration integer)")
    syms = {}
    for name, mangled, grid, wg, vgpr, dur in launches:
        kid = syms.setdefault((name, mangled), len(syms) + 1)
        con.execute("insert into kernels values (?, ?, ?, ?, ?, ?)", (name, kid, grid, wg, vgpr, dur))
    for (name, mangled), kid in syms.items():
        con.execute("insert into kernel_symbols values (?, ?)", (kid, mangled))
    con.commit()
    con.close()


def _pmc_db(path, counter, rows):
    con = sqlite3.connect(path)
    con.execute("create table kernel_symbols (kernel_id integer, kernel_name text)")
    con.execute("create table counters_collection (kernel_name text, kernel_id integer, grid_size integer, "
                "counter_name text, value real)")
    for kid, (name, grid, value) in enumerate(rows, start=1):
        con.execute("insert into kernel_symbols values (?, ?)", (kid, ""))
        con.execute("insert into counters_collection values (?, ?, ?, ?, ?)", (name, kid, grid, counter, value))
    con.commit()
    con.close()


SWEEP = "void lbm::k_sweep<lbm::D3Q19, 1, double, 1>(double const*, double*, unsigned char const*, int)"
SWEEP16 = "_ZN3lbm7k_sweepINS_5D3Q27ELi8EDF16_Li1EEEvPKT1_PS2_PKhPKNS_7StorageIS2_E1RENS_3GeoENS_13CollideParamsISA_EEi"
COPY = "void lbm::(anonymous namespace)::k_copy_q<unsigned long, 19, 1>(unsigned long const*, unsigned long*, long)"


def test_trace_summary_groups_by_kernel_and_grid(tmp_path):
    d = tmp_path / "trace"
    d.mkdir()
    _trace_db(str(d / "trace_results.db"), [
        (SWEEP, "", 16777216, 256, 40, 900), (SWEEP, "", 16777216, 256, 40, 1100),
        (SWEEP, "", 2097152, 128, 40, 100),
        ("bool _Accum", SWEEP16, 134217728, 512, 24, 2800),
    ])
    out = bench.trace_summary(str(d)).splitlines()
    rows = {l.split("  ")[-1].strip(): l.split() for l in out[1:]}
    big = [l.split() for l in out[1:] if l.endswith("k_sweep<D3Q19, TRT, double, NT>") and " 16777216 " in l][0]
    assert big[:4] == ["2", "1000", "900", "1100"]
    assert big[6] == "80"          # VGPRs allocated: twice rocprofv3's granule-of-4 figure
    small = [l.split() for l in out[1:] if " 2097152 " in l][0]
    assert small[:2] == ["1", "100"]
    assert any(k == "k_sweep<D3Q27, MRT_UNIT, f16, NT>" for k in rows), rows   # from the mangled symbol


def test_pmc_summary_calibrates_on_copy_kernels(tmp_path):
    n = 1 << 20
    copy_bytes = 19 * 8 * n
    fetch, write = tmp_path / "fetch", tmp_path / "write"
    fetch.mkdir()
    write.mkdir()
    # the copy reads copy_bytes, FETCH_SIZE counts half of it; WRITE_SIZE counts all
    _pmc_db(str(fetch / "fetch_results.db"), "FETCH_SIZE",
            [(COPY, n, copy_bytes / 2 / 1024), (SWEEP, n, 1.01 * copy_bytes / 2 / 1024)])
    _pmc_db(str(write / "write_results.db"), "WRITE_SIZE",
            [(COPY, n, copy_bytes / 1024), (SWEEP, n, copy_bytes / 1024)])
    out = bench.pmc_summary(str(fetch), str(write))
    assert "fetch 2.0000" in out and "write 1.0000" in out
    line = [l for l in out.splitlines() if l.endswith("k_sweep<D3Q19, TRT, double, NT>")][0].split()
    assert float(line[0]) == pytest.approx(1.01 * copy_bytes / 2 / 1024, rel=1e-6)


def test_pmc_summary_needs_a_copy_kernel(tmp_path):
    fetch, write = tmp_path / "fetch", tmp_path / "write"
    fetch.mkdir()
    write.mkdir()
    _pmc_db(str(fetch / "fetch_results.db"), "FETCH_SIZE", [(SWEEP, 64, 1.0)])
    _pmc_db(str(write / "write_results.db"), "WRITE_SIZE", [(SWEEP, 64, 1.0)])
    with pytest.raises(SystemExit, match="nothing to calibrate"):
        bench.pmc_summary(str(fetch), str(write))
