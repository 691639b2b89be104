"""Host-side tools: the profile summariser, the benchmark's command line, the
synthetic input generators."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _write(path, header, rows):
    with open(path, "w") as f:
        f.write(",".join(f'"{h}"' for h in header) + "\n")
        for r in rows:
            f.write(",".join(f'"{x}"' if isinstance(x, str) else str(x) for x in r) + "\n")


def test_profsum_scales_counters_by_the_copy_kernel(tmp_path):
    from paper_1804_10120_amd import profsum
    n = 1000
    trace, fetch, write, out = (tmp_path / d for d in ("trace", "fetch", "write", "out"))
    for d in (trace, fetch, write):
        d.mkdir()
    bwd = "void tl::k_points<tl::OpChainBwd, 256, 1, true>(tl::KArgs, long, long, int)"
    fwd = "void tl::k_points<tl::OpChain, 256, 1, true>(tl::KArgs, long, long, int)"
    copy = "tl::k_copy(double const*, double*, long)"
    _write(trace / "t_kernel_stats.csv", ["Name", "Calls", "TotalDurationNs", "AverageNs",
                                          "Percentage"], [[bwd, 2, 200.0, 100.0, 60.0]])
    _write(trace / "t_kernel_trace.csv", ["Kernel_Name", "Grid_Size_X", "Start_Timestamp",
                                          "End_Timestamp", "VGPR_Count", "Accum_VGPR_Count"],
           [[bwd, 1024, 0, 100, 89, 0], [bwd, 1024, 200, 300, 89, 0]])
    copy_doubles = 4096
    hdr = ["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]
    # the counter sees half the fetched bytes and all the written ones
    _write(fetch / "f_counter_collection.csv", hdr,
           [[copy, 2048, "FETCH_SIZE", 8 * copy_doubles / 1024 / 2],
            [bwd, 1024, "FETCH_SIZE", 8 * 40 * n / 1024 / 2],
            [fwd, 1024, "FETCH_SIZE", 8 * 43 * n / 1024 / 2]])
    _write(write / "w_counter_collection.csv", hdr,
           [[copy, 2048, "WRITE_SIZE", 8 * copy_doubles / 1024],
            [bwd, 1024, "WRITE_SIZE", 8 * 43 * n / 1024],
            [fwd, 1024, "WRITE_SIZE", 8 * 6 * n / 1024]])
    r = subprocess.run([sys.executable, "-m", "paper_1804_10120_amd.profsum", "--trace",
                        str(trace), "--fetch", str(fetch), "--write", str(write), "--cmd", "x",
                        "--points", str(n), "--copy-doubles", str(copy_doubles), "--workload",
                        "w", "--out", str(out)], cwd=ROOT, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    rec = {}
    for line in open(out / "pmc_dtg_chain_bwd.md"):
        if ":" in line and not line.startswith(("#", "|", " ")):
            k, v = line.split(":", 1)
            rec[k.strip()] = v.strip()
    assert float(rec["traffic_bytes_per_launch"]) == 8 * 83 * n
    assert rec["sources_sha256"] == profsum.sources_sha256()
    assert "| 2 | 0.10 |" in open(out / "kernel_stats_w.md").read()


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_synthetic_fields_are_seeded_and_in_range():
    from paper_1804_10120_amd.synth import domain_edges, make_expr_inputs, make_fields
    a, b = make_fields(1000, seed=3), make_fields(1000, seed=3)
    assert all(np.array_equal(a[k], b[k]) for k in a)
    c = make_fields(1000, seed=3, fields=("dg",))
    assert np.array_equal(c["dg"], a["dg"])            # a field does not depend on the others
    g = a["g"]
    full = np.array([[g[0], g[1], g[2]], [g[1], g[3], g[4]], [g[2], g[4], g[5]]])
    ev = np.linalg.eigvalsh(full.transpose(2, 0, 1))
    assert ev.min() >= 0.7 - 1e-12 and ev.max() <= 1.3 + 1e-12
    assert 0.5 <= a["alpha"].min() and a["alpha"].max() <= 1.5
    assert np.abs(a["beta"]).max() <= 0.5
    e = domain_edges(256)
    assert e.min() >= 8 and e.max() <= 48 and len(e) == 256
    x = make_expr_inputs("kij", 100, seed=1)
    assert [v.shape[0] for v in x] == [1, 6, 3] and x[0].min() >= 0.5


def test_record_is_per_thread():
    """A recording on one thread does not capture another thread's calls."""
    import threading
    from paper_1804_10120_amd import ops
    seen = {}

    def other():
        seen["other"] = ops._recording()

    with ops.record() as calls:
        t = threading.Thread(target=other)
        t.start()
        t.join()
        assert ops._recording() is calls
    assert seen["other"] is None
    assert ops._recording() is None


def test_autotune_cache_roundtrip(tmp_path, monkeypatch):
    """The tuning cache: atomic writes leave no temporary file, and a read after
    a new write sees the new contents (reads are memoised per file version)."""
    from paper_1804_10120_amd import autotune
    path = tmp_path / "sub" / "tune.json"
    monkeypatch.setenv("TLMI_TUNE_CACHE", str(path))
    assert autotune.load_cache() == {}
    autotune.save_cache({"k|gfx950|log2n=21": {"tune": {"block": 256}}})
    assert autotune.load_cache()["k|gfx950|log2n=21"]["tune"] == {"block": 256}
    c = autotune.load_cache()
    c["other"] = {"tune": {"block": 64}}
    assert "other" not in autotune.load_cache()      # callers get a copy
    autotune.save_cache(c)
    assert autotune.load_cache()["other"]["tune"] == {"block": 64}
    assert sorted(p.name for p in path.parent.iterdir()) == ["tune.json"]


def test_traffic_record_goes_stale_when_the_build_inputs_change(tmp_path):
    """The committed counter figure is reported only while every input of the
    library's machine code is unchanged: a kernel source, a generated kernel,
    a public header (the hash also covers the compiler flags)."""
    import shutil
    sys.path.insert(0, ROOT)
    import bench
    from paper_1804_10120_amd import profsum
    pkg = os.path.basename(os.path.dirname(profsum.__file__))
    root = tmp_path / "repo"
    shutil.copytree(os.path.join(ROOT, pkg, "csrc"), root / pkg / "csrc")
    shutil.copytree(os.path.join(ROOT, "include"), root / "include")
    (root / "profiles").mkdir()
    n = 4096

    def write_record():
        (root / "profiles" / "pmc_dtg_chain_bwd.md").write_text(
            f"# x\n\nkernel: dtg_chain_bwd\npoints: {n}\n"
            f"sources_sha256: {profsum.sources_sha256(str(root))}\n"
            f"traffic_bytes_per_launch: 1234\n")

    write_record()
    assert bench.traffic_record("dtg_chain_bwd", n, root=str(root)) == 1234.0
    assert bench.traffic_record("dtg_chain_bwd", n + 1, root=str(root)) is None
    for rel in ("include/tl.h", f"{pkg}/csrc/generated/tlg_kernels.hip",
                f"{pkg}/csrc/tl_stream.hpp"):
        write_record()
        with open(root / rel, "a") as f:
            f.write("\n// edited\n")
        assert bench.traffic_record("dtg_chain_bwd", n, root=str(root)) is None, rel


def test_threaded_oracle_equals_the_serial_oracle():
    """The tests' threaded runner of the oracle (point ranges on host threads,
    joined in point order) gives bitwise the serial oracle's results."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import oracle
    import oracle_par
    from paper_1804_10120_amd.synth import make_expr_inputs, make_fields
    n = 1000
    f = make_fields(n, seed=77)
    keys = oracle_par.KEYS
    assert np.array_equal(oracle_par.over_points(oracle.dtg_chain, *[f[k] for k in keys],
                                                 chunk=97),
                          oracle.dtg_chain(*[f[k] for k in keys]))
    par = oracle_par.over_points(lambda *x: oracle.dtg_chain_vjp(tuple(x[:6]), x[6]),
                                 *[f[k] for k in keys], f["W"], chunk=131)
    ser = oracle.dtg_chain_vjp(tuple(f[k] for k in keys), f["W"])
    assert set(par) == set(ser) and all(np.array_equal(par[k], ser[k]) for k in ser)
    xs = make_expr_inputs("contract2", n, seed=5)
    assert np.array_equal(oracle_par.expr("contract2", *xs), oracle.expr("contract2", *xs))


def test_profsum_labelled_dispatches(tmp_path):
    """Dispatches renamed after bench.py's labels are grouped per label, with
    the algorithmic GB/s of the average duration."""
    from paper_1804_10120_amd import profsum
    trace = tmp_path / "trace"
    trace.mkdir()
    hdr = ["Kernel_Name", "Grid_Size_X", "Start_Timestamp", "End_Timestamp", "VGPR_Count",
           "Accum_VGPR_Count"]
    n = 262144
    _write(trace / "t_kernel_trace.csv", hdr,
           [["c2 dtg_chain n=262144", n, 0, 20000, 62, 0],
            ["c2 dtg_chain n=262144", n, 30000, 40000, 62, 0],
            ["c5 dtg_chain_bwd n=262144 ppt2_b512", n // 4, 0, 30000, 166, 0],
            ["c4 dtg_chain n=262144 4 launches", n // 4, 0, 5000, 62, 0],
            ["c4 dtg_chain n=262144 4 launches", n // 4, 9000, 16000, 62, 0],
            ["void tl::k_copy(double const*, double*, long)", 1024, 0, 5, 12, 0]])
    rows = profsum.labelled_dispatches(str(trace))
    assert [r["label"] for r in rows] == ["c2 dtg_chain n=262144",
                                          "c4 dtg_chain n=262144 4 launches",
                                          "c5 dtg_chain_bwd n=262144 ppt2_b512"]
    a, s, b = rows
    # n points over 4 launches of 6 us on average: 24 us per pass
    assert s["calls"] == 2 and abs(s["GB_s"] - 392 * n / 24000) < 1e-9
    assert a["calls"] == 2 and a["avg_ns"] == 15000 and a["min_ns"] == 10000
    assert abs(a["GB_s"] - 392 * n / 15000) < 1e-9 and b["variant"] == "ppt2_b512"
    assert abs(b["frac"] - 664 * n / 30000 / 8000) < 1e-12
