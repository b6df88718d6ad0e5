"""Host-side checks of the C ABI (no GPU needed).

* The library loads and exports every function include/concord.h declares.
* concord_schedule (the closed form the kernels use) equals the oracle's
  round-robin table (the circle method of Section 3.2, built seat by seat)
  bit for bit, slot order included.
* Invalid arguments are rejected before any device work.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "concord.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(concord_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2106_09382_amd import _lib
    return _lib.load()


def test_header_declares_the_entry_points():
    names = _declared_functions()
    for want in ("concord_fit", "concord_fit_ex", "concord_gram", "concord_schedule",
                 "concord_strerror", "concord_version"):
        assert want in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared_functions():
        assert hasattr(lib, name), name


@pytest.mark.parametrize("p", list(range(1, 130)) + [255, 256, 1000, 1001, 2000, 2001])
def test_closed_form_schedule_matches_oracle_table(p):
    from paper_2106_09382_amd import _lib
    assert np.array_equal(_lib.schedule(p), oracle.round_robin(p))


def test_schedule_rejects_bad_p(lib):
    buf = (ctypes.c_int32 * 4)()
    assert lib.concord_schedule(0, buf) == -1
    assert lib.concord_schedule(-3, buf) == -1
    assert lib.concord_schedule(4, None) == -1


def test_strerror_covers_codes(lib):
    for c in (0, 1, -1, -2, -3, -4, -5, -6, -7):
        s = lib.concord_strerror(c).decode()
        assert s and s != "unknown status code"
    assert lib.concord_strerror(99).decode() == "unknown status code"
    assert b"gfx950" in lib.concord_version()


def _fit(lib, **kw):
    from paper_2106_09382_amd import _lib
    a = dict(kind=0, X=ctypes.c_void_p(0x1000), n=0, p=8, lam=0.1, tol=1e-6, maxit=10, dt=1,
             omega0=None, omega=ctypes.c_void_p(0x2000))
    a.update(kw)
    info = _lib.ConcordInfo()
    rc = lib.concord_fit(a["kind"], a["X"], a["n"], a["p"], a["lam"], a["tol"], a["maxit"],
                         a["dt"], a["omega0"], a["omega"], ctypes.byref(info), None)
    return rc, info


@pytest.mark.parametrize("kw", [
    dict(X=None), dict(omega=None), dict(p=0), dict(p=-5), dict(p=50000),
    dict(lam=-0.1), dict(lam=float("nan")), dict(lam=float("inf")),
    dict(tol=0.0), dict(tol=-1.0), dict(tol=float("nan")), dict(maxit=0),
    dict(dt=7), dict(kind=5), dict(kind=1, n=0),
])
def test_invalid_arguments_return_einval(lib, kw):
    rc, info = _fit(lib, **kw)
    assert rc == -1 and info.status == -1


@pytest.mark.parametrize("kw", [
    dict(X=None), dict(omega=None), dict(p=0), dict(p=50000), dict(lam=-0.1),
    dict(tol=0.0), dict(maxit=0), dict(dt=7), dict(kind=5), dict(kind=1, n=0),
])
def test_noalloc_invalid_arguments_return_einval(lib, kw):
    """concord_fit_noalloc checks its arguments as concord_fit does, before
    it looks up its scratch on the device."""
    from paper_2106_09382_amd import _lib
    a = dict(kind=0, X=ctypes.c_void_p(0x1000), n=0, p=8, lam=0.1, tol=1e-6, maxit=10, dt=1,
             omega0=None, omega=ctypes.c_void_p(0x2000))
    a.update(kw)
    info = _lib.ConcordInfo()
    info.sweeps = 77
    rc = lib.concord_fit_noalloc(a["kind"], a["X"], a["n"], a["p"], a["lam"], a["tol"],
                                 a["maxit"], a["dt"], a["omega0"], a["omega"],
                                 ctypes.byref(info), None)
    assert rc == -1 and info.status == -1 and info.sweeps == 0


def test_noalloc_scratch_size_matches_the_header():
    from paper_2106_09382_amd import _lib
    text = open(HEADER).read()
    m = re.search(r"#define CONCORD_NOALLOC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", text)
    assert m, "CONCORD_NOALLOC_SCRATCH_BYTES not found"
    assert int(m.group(1)) << int(m.group(2)) == _lib.NOALLOC_SCRATCH_BYTES
    assert "CONCORD_ESCRATCH = -7" in text and _lib.ESCRATCH == -7


@pytest.mark.parametrize("rows,cols,threads", [(32, 8, 512), (16, 16, 256), (1, 1, 64)])
def test_rows_per_thread_cap_returns_elaunch(lib, rows, cols, threads):
    """A workgroup holds at most two rows of W per thread, so a launch of
    `rows` row groups of `threads` threads serves p <= 2 * threads * rows; one
    more row is refused with CONCORD_ELAUNCH while the launch shape is chosen,
    before any device work (the input pointers here are not device memory)."""
    from paper_2106_09382_amd import _lib
    cap = 2 * threads * rows
    opts = _lib.ConcordOptions()
    opts.row_groups, opts.col_slices, opts.block_threads = rows, cols, threads
    info = _lib.ConcordInfo()
    for dt in (0, 1):
        rc = lib.concord_fit_ex(0, ctypes.c_void_p(0x1000), 0, cap + 1, 0.1, 1e-6, 10, dt, None,
                                ctypes.c_void_p(0x2000), ctypes.byref(info), None,
                                ctypes.byref(opts))
        assert rc == _lib.ELAUNCH


@pytest.mark.parametrize("dt,threads,wl,want", [
    (0, 1088, 0, "EINVAL"),    # FP32: at most 1024 threads
    (1, 832, 0, "EINVAL"),     # FP64: at most 768 threads
    (1, 1024, 0, "EINVAL"),
    (0, 1024, 1, "EINVAL"),    # a wide workgroup keeps W in HBM
    (0, 1024, 0, "ELAUNCH"),   # one row per thread: p = rows x threads + 1 does not fit
    (1, 768, 0, "ELAUNCH"),
])
def test_wide_workgroups_are_checked_before_device_work(lib, dt, threads, wl, want):
    """Workgroups of more than 512 threads (the wide sweep kernel) hold one row
    of W per thread with W in HBM; requests outside that are refused while
    the launch shape is chosen (the pointers here are not device memory)."""
    from paper_2106_09382_amd import _lib
    rows = 32
    opts = _lib.ConcordOptions()
    opts.row_groups, opts.col_slices, opts.block_threads, opts.w_in_lds = rows, 8, threads, wl
    info = _lib.ConcordInfo()
    rc = lib.concord_fit_ex(0, ctypes.c_void_p(0x1000), 0, rows * threads + 1, 0.1, 1e-6, 10, dt,
                            None, ctypes.c_void_p(0x2000), ctypes.byref(info), None,
                            ctypes.byref(opts))
    assert rc == getattr(_lib, want)


@pytest.mark.parametrize("dt", [0, 1])
def test_joint_wide_workgroups_stop_at_768_threads(lib, dt):
    """The joint kernel's wide form reaches 768 threads in both precisions;
    1024 is refused before any device work."""
    from paper_2106_09382_amd import _lib
    opts = _lib.ConcordOptions()
    opts.block_threads = 1024
    rc, _ = _fit_joint(lib, opts=opts, dt=dt)
    assert rc == _lib.EINVAL


def test_gram_rejects_bad_sizes(lib):
    assert lib.concord_gram(None, 10, 10, 1, ctypes.c_void_p(0x10), None) == -1
    assert lib.concord_gram(ctypes.c_void_p(0x10), 0, 10, 1, ctypes.c_void_p(0x10), None) == -1
    assert lib.concord_gram(ctypes.c_void_p(0x10), 10, 10, 3, ctypes.c_void_p(0x10), None) == -1


def _fit_batched(lib, B=2, L=3, **kw):
    from paper_2106_09382_amd import _lib
    vp = ctypes.c_void_p
    a = dict(B=B, kind=0, X=(vp * B)(*([0x1000] * B)), n=None, p=(ctypes.c_int64 * B)(*([8] * B)),
             L=L, lam=(ctypes.c_double * (B * L))(*([0.1] * (B * L))), tol=1e-6, maxit=10, dt=1,
             omega=(vp * (B * L))(*([0x2000] * (B * L))))
    a.update(kw)
    return lib.concord_fit_batched(a["B"], a["kind"], a["X"], a["n"], a["p"], a["L"], a["lam"],
                                   a["tol"], a["maxit"], a["dt"], a["omega"], None, None)


def test_batched_invalid_arguments_return_einval(lib):
    vp = ctypes.c_void_p
    assert _fit_batched(lib, B=0) == -1
    assert _fit_batched(lib, L=0) == -1
    assert _fit_batched(lib, X=None) == -1
    assert _fit_batched(lib, p=None) == -1
    assert _fit_batched(lib, lam=None) == -1
    assert _fit_batched(lib, omega=None) == -1
    assert _fit_batched(lib, kind=1, n=None) == -1
    assert _fit_batched(lib, kind=1, n=(ctypes.c_int64 * 2)(4, 0)) == -1
    assert _fit_batched(lib, p=(ctypes.c_int64 * 2)(8, 0)) == -1
    assert _fit_batched(lib, X=(vp * 2)(0x1000, None)) == -1
    assert _fit_batched(lib, lam=(ctypes.c_double * 6)(0.5, 0.2, 0.1, 0.5, float("nan"), 0.1)) == -1
    assert _fit_batched(lib, lam=(ctypes.c_double * 6)(0.5, 0.2, 0.1, 0.5, -1.0, 0.1)) == -1
    assert _fit_batched(lib, omega=(vp * 6)(0x2000, 0x2000, 0x2000, 0x2000, 0x2000, None)) == -1
    assert _fit_batched(lib, tol=0.0) == -1
    assert _fit_batched(lib, maxit=0) == -1
    assert _fit_batched(lib, L=3, maxit=(1 << 23)) == -1  # L * maxit > 2^24
    assert _fit_batched(lib, dt=5) == -1


def _fit_batched_ex(lib, opts, B=2, p=8, dt=1):
    from paper_2106_09382_amd import _lib
    vp = ctypes.c_void_p
    L = 3
    return lib.concord_fit_batched_ex(
        B, 0, (vp * B)(*([0x1000] * B)), None, (ctypes.c_int64 * B)(*([p] * B)), L,
        (ctypes.c_double * (B * L))(*([0.1] * (B * L))), 1e-6, 10, dt,
        (vp * (B * L))(*([0x2000] * (B * L))), None, None, ctypes.byref(opts))


@pytest.mark.parametrize("dt,threads,want", [(0, 1088, "EINVAL"), (1, 832, "EINVAL"),
                                             (1, 1024, "EINVAL")])
def test_batched_wide_workgroups_are_bounded(lib, dt, threads, want):
    """The batch's workgroups reach 1024 threads in FP32 and 768 in FP64
    (one row per thread); wider is refused before any device work."""
    from paper_2106_09382_amd import _lib
    opts = _lib.ConcordBatchOptions()
    opts.block_threads = threads
    assert _fit_batched_ex(lib, opts, dt=dt) == getattr(_lib, want)


def test_batched_wide_workgroups_hold_one_row_per_thread(lib):
    """With 768 threads a workgroup holds at most 768 rows: a problem of 1537
    rows on 2 workgroups is refused before any device work (512-thread
    workgroups, two rows per thread, would hold it)."""
    from paper_2106_09382_amd import _lib
    opts = _lib.ConcordBatchOptions()
    opts.block_threads = 768
    pw = (ctypes.c_int32 * 2)(2, 2)
    opts.problem_workgroups = pw
    assert _fit_batched_ex(lib, opts, p=1537) == _lib.EINVAL


def test_autotune_plan_deals_by_work():
    from paper_2106_09382_amd import autotune
    ps = [200, 1500, 3000, 50]
    G = autotune.plan(ps, [1.0, 1.0, 1.0, 1.0], 40)
    assert sum(G) <= 40 and all(g >= autotune.min_workgroups(p) for g, p in zip(G, ps))
    assert all(g * 8 <= p or g == autotune.min_workgroups(p) for g, p in zip(G, ps))
    heavy = autotune.plan(ps, [1.0, 10.0, 1.0, 1.0], 40)
    assert heavy[1] > G[1]
    infos = [[{"sweep_ms": 5.0, "row_groups": g, "col_slices": 1}] for g in G]
    assert sum(autotune.plan_from_infos(ps, infos, 40)) <= 40
    with pytest.raises(ValueError):
        autotune.plan([5000] * 10, [1.0] * 10, 12)
    # with column slices a count stays a multiple of its problem's slices
    S = autotune.plan([3000, 2000, 400], [3.0, 2.0, 1.0], 40, slices=[2, 4, 1])
    assert S[0] % 2 == 0 and S[1] % 4 == 0 and sum(S) <= 40
    assert S[0] >= autotune.min_workgroups(3000, 512, 2)


def test_autotune_search_keeps_what_measures_faster():
    """The search on a model batch whose per-problem time is work / workgroups,
    where two column slices halve the work of the large problems and two
    columns per lane slow everything: it must pick the slices for exactly
    the large problems and keep four columns per lane."""
    from paper_2106_09382_amd import autotune
    ps = [300, 800, 2500, 3000]
    base = {300: 1.0, 800: 4.0, 2500: 30.0, 3000: 40.0}
    calls = []

    def run(pw, pc, cpl):
        calls.append((pw, pc, cpl))
        pw = pw or [8] * len(ps)
        pc = pc or [1] * len(ps)
        infos = []
        for p, g, c in zip(ps, pw, pc):
            work = base[p] * (0.5 if (c == 2 and p >= 2000) else (1.5 if c == 2 else 1.0))
            work *= 1.2 if cpl == 2 else 1.0
            infos.append([{"sweep_ms": work / g, "row_groups": g // c, "col_slices": c}])
        return infos, max(r[0]["sweep_ms"] for r in infos)

    best = autotune.search(run, ps, 64)
    # a launch too small to give every problem two slices: only the heaviest
    # is tried with them (minimum 2 workgroups each, 4 with two slices)
    tried = []

    def run_tight(pw, pc, cpl):
        tried.append(pc)
        pw = pw or [2, 2, 3, 4]
        pc = pc or [1] * 4
        infos = [[{"sweep_ms": (4.0 if b == 3 else 1.0) / g, "row_groups": g // c,
                   "col_slices": c}] for b, (g, c) in enumerate(zip(pw, pc))]
        return infos, max(r[0]["sweep_ms"] for r in infos)

    tight = autotune.search(run_tight, [1500, 1500, 1500, 1500], 11)
    assert [1, 1, 1, 2] in tried
    assert sum(tight["problem_workgroups"]) <= 11
    assert all(g % c == 0 for g, c in zip(tight["problem_workgroups"],
                                          tight["problem_col_slices"]))
    C = best["problem_col_slices"]
    assert C[2] == 2 and C[3] == 2 and C[0] == 1 and C[1] == 1
    assert best["cols_per_lane"] == 4
    assert sum(best["problem_workgroups"]) <= 64
    for p, g, c in zip(ps, best["problem_workgroups"], C):
        assert g % c == 0 and -(-p // (g // c)) <= 1024
    assert best["wall_s"] == min(t["wall_s"] for t in best["trials"])
    assert calls[0] == (None, None, 4) and len(calls) == len(best["trials"])
    # the plan returned is one that ran, as it ran (no list changed afterwards)
    assert any(t["problem_workgroups"] == best["problem_workgroups"]
               and t["problem_col_slices"] == best["problem_col_slices"]
               and t["cols_per_lane"] == best["cols_per_lane"]
               and t["wall_s"] == best["wall_s"] for t in best["trials"])

    # a model where the slices lower the large problems' own times but the
    # batch as a whole runs slower with them: the one-slice plan must come
    # back exactly as it was run, although the per-problem choice picked slices
    def run_slow(pw, pc, cpl):
        infos, wall = run(pw, pc, cpl)
        return infos, wall * (3.0 if pc and any(c == 2 for c in pc) else 1.0)

    slow = autotune.search(run_slow, ps, 64)
    assert slow["problem_col_slices"] == [1] * len(ps)
    assert any(t["problem_workgroups"] == slow["problem_workgroups"]
               and t["problem_col_slices"] == slow["problem_col_slices"]
               and t["wall_s"] == slow["wall_s"] for t in slow["trials"])


def test_autotune_search_tries_wide_workgroups():
    """With wide_threads, the search also runs wide workgroups (one row per
    thread) dealt by the measured work, and keeps them only if the batch runs
    faster; the wide plan gives every problem at least ceil(p / threads)
    workgroups of one slice."""
    from paper_2106_09382_amd import autotune
    assert autotune.max_rows(512) == 1024 and autotune.max_rows(1024) == 1024
    assert autotune.min_workgroups(2000, 768) == 3 and autotune.min_workgroups(2000, 512) == 2
    ps = [300, 800, 2500, 3000]
    base = {300: 1.0, 800: 4.0, 2500: 30.0, 3000: 40.0}

    def model(speed):
        seen = []

        def run(pw, pc, cpl, threads=512):
            seen.append(threads)
            pw = pw or [8] * len(ps)
            pc = pc or [1] * len(ps)
            f = speed if threads > 512 else 1.0
            infos = [[{"sweep_ms": base[p] * f / g, "row_groups": g // c, "col_slices": c}]
                     for p, g, c in zip(ps, pw, pc)]
            return infos, max(r[0]["sweep_ms"] for r in infos)
        return run, seen

    run, seen = model(0.8)
    best = autotune.search(run, ps, 64, slice_options=(), wide_threads=1024)
    assert 1024 in seen and best["block_threads"] == 1024
    assert best["problem_col_slices"] == [1] * len(ps)
    for p, g in zip(ps, best["problem_workgroups"]):
        assert g >= autotune.min_workgroups(p, 1024)
    assert sum(best["problem_workgroups"]) <= 64
    run, seen = model(1.5)
    best = autotune.search(run, ps, 64, slice_options=(), wide_threads=1024)
    assert 1024 in seen and best["block_threads"] == 512
    assert all(t["block_threads"] in (512, 1024) for t in best["trials"])


def _fit_joint(lib, opts=None, **kw):
    from paper_2106_09382_amd import _lib
    vp = ctypes.c_void_p
    a = dict(kind=0, X1=vp(0x1000), X2=vp(0x3000), n1=0, n2=0, p=8, lam1=0.1, lam2=0.05,
             tol=1e-6, maxit=10, dt=1, o01=None, o02=None, o1=vp(0x2000), o2=vp(0x4000))
    a.update(kw)
    info = _lib.ConcordJointInfo()
    rc = lib.concord_fit_joint_ex(a["kind"], a["X1"], a["X2"], a["n1"], a["n2"], a["p"],
                                  a["lam1"], a["lam2"], a["tol"], a["maxit"], a["dt"], a["o01"],
                                  a["o02"], a["o1"], a["o2"], ctypes.byref(info), None,
                                  ctypes.byref(opts) if opts is not None else None)
    return rc, info


@pytest.mark.parametrize("kw", [
    dict(X1=None), dict(X2=None), dict(o1=None), dict(o2=None), dict(o2=ctypes.c_void_p(0x2000)),
    dict(p=0), dict(p=50000), dict(lam1=-0.1), dict(lam2=-0.1), dict(lam2=float("nan")),
    dict(lam2=float("inf")), dict(tol=0.0), dict(maxit=0), dict(dt=4), dict(kind=3),
    dict(kind=1, n1=10, n2=0),
])
def test_joint_invalid_arguments_return_einval(lib, kw):
    rc, info = _fit_joint(lib, **kw)
    assert rc == -1 and info.status == -1


@pytest.mark.parametrize("field", ["active_set", "w_out", "device_timestamps"])
def test_joint_rejects_single_solve_options(lib, field):
    from paper_2106_09382_amd import _lib
    opts = _lib.ConcordOptions()
    setattr(opts, field, 1)
    rc, _ = _fit_joint(lib, opts=opts)
    assert rc == -1


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes structures have the C header's sizes and field offsets
    (a small C program compiled with gcc prints them)."""
    from paper_2106_09382_amd import _lib
    structs = {"concord_info": _lib.ConcordInfo, "concord_joint_info": _lib.ConcordJointInfo,
               "concord_options": _lib.ConcordOptions,
               "concord_batch_options": _lib.ConcordBatchOptions}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "concord.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True,
                               check=True).stdout.splitlines():
        c, f, v = line.split()
        got[(c, f)] = int(v)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_profiling_driver_rejects_bad_runs_before_device_work():
    """concord_bench: an unknown flag prints the usage and exits 2; runs joined
    by --then stop at the first one that fails, so the copy after it never
    starts (it would print its size)."""
    import subprocess
    from paper_2106_09382_amd import build
    if not os.path.exists(build.BENCH):
        pytest.skip("concord_bench is not built")
    r = subprocess.run([build.BENCH, "--bogus", "--then", "--copy", "1"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "usage: concord_bench" in r.stderr and "--then RUN" in r.stderr
    assert "copy_bytes" not in r.stdout
    r = subprocess.run([build.BENCH, "--y", "/nonexistent", "--n", "0", "--p", "5"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2 and "usage: concord_bench" in r.stderr
