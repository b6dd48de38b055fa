"""Host-side checks of libpsdproj: it loads, exports every declared entry point, keeps the
struct layout of include/psdproj.h, and validates descriptors without touching a device."""
import ctypes
import os
import re
import shutil
import subprocess
import tempfile

import pytest

import paper_2410_19208_amd as pp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "psdproj.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(psdproj_[a-z_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported_and_bound():
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(pp.lib, name), name
    assert set(names) == set(pp.EXPORTED)


def test_abi_version():
    assert pp.psdproj_abi_version() == 1


@pytest.mark.skipif(not shutil.which("gcc"), reason="gcc not available")
def test_struct_layout_matches_header():
    prog = r"""
#include <stdio.h>
#include <stddef.h>
#include "psdproj.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu\n", sizeof(psdproj_desc), offsetof(psdproj_desc, seed),
         offsetof(psdproj_desc, alpha), offsetof(psdproj_desc, alpha_iters), offsetof(psdproj_desc, flags));
  printf("%zu %zu %zu\n", sizeof(psdproj_result), offsetof(psdproj_result, alpha_used), offsetof(psdproj_result, sigma2));
  printf("%zu %zu %zu\n", sizeof(psdproj_layout), offsetof(psdproj_layout, omega), offsetof(psdproj_layout, total));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "l.c")
        open(src, "w").write(prog)
        exe = os.path.join(d, "l")
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    d = [int(x) for x in out[0].split()]
    r = [int(x) for x in out[1].split()]
    lay = [int(x) for x in out[2].split()]
    assert d == [ctypes.sizeof(pp.Desc), pp.Desc.seed.offset, pp.Desc.alpha.offset, pp.Desc.alpha_iters.offset,
                 pp.Desc.flags.offset]
    assert r == [ctypes.sizeof(pp.Result), pp.Result.alpha_used.offset, pp.Result.sigma2.offset]
    assert lay == [ctypes.sizeof(pp.Layout), pp.Layout.omega.offset, pp.Layout.total.offset]


def plan_status(**kw):
    base = dict(n=100, k=10, p=5, q=1, variant=pp.PLAIN, precision=pp.FP32, seed=0, alpha=0.0, alpha_iters=10,
                flags=0)
    base.update(kw)
    d = pp.Desc(base["n"], base["k"], base["p"], base["q"], base["variant"], base["precision"], base["seed"],
                base["alpha"], base["alpha_iters"], base["flags"])
    h = ctypes.c_void_p()
    ws = ctypes.c_size_t()
    st = pp.lib.psdproj_plan(ctypes.byref(d), ctypes.byref(h), ctypes.byref(ws))
    if st == 0:
        pp.lib.psdproj_plan_destroy(h)
    return st, ws.value


@pytest.mark.parametrize("kw", [
    dict(k=0), dict(p=-1), dict(k=96, p=5), dict(q=-1), dict(q=17), dict(variant=2), dict(precision=3),
    dict(flags=4), dict(flags=0x80000000), dict(n=0), dict(n=300, k=250, p=10),
    dict(variant=pp.SCALED, alpha=float("nan")), dict(variant=pp.SCALED, alpha=float("inf")),
    dict(variant=pp.SCALED, alpha=0.0, alpha_iters=0), dict(variant=pp.SCALED, alpha=-1.0, alpha_iters=1001),
])
def test_plan_rejects_invalid(kw):
    assert plan_status(**kw)[0] == pp.E_INVALID


@pytest.mark.parametrize("kw", [
    dict(), dict(k=1, p=0, q=0, n=1), dict(n=7, k=5, p=2), dict(variant=pp.SCALED, alpha=2.0),
    dict(variant=pp.SCALED, alpha=0.0, alpha_iters=1), dict(precision=pp.FP64), dict(precision=pp.BF16X3),
    dict(n=20000, k=200, p=20, q=1, precision=pp.BF16X3), dict(n=4096, k=246, p=10),
])
def test_plan_accepts_valid(kw):
    st, ws = plan_status(**kw)
    assert st == pp.OK and ws > 0


def test_workspace_grows_with_n_and_layout_is_consistent():
    small = plan_status(n=1000)[1]
    big = plan_status(n=4000)[1]
    assert big > small
    plan, ws = pp.psdproj_plan(4000, 100, 10, 1, pp.SCALED, pp.BF16X3)
    try:
        L = pp.psdproj_plan_layout(plan)
        assert L.r == 110 and L.r_pad % 32 == 0 and L.r_pad >= 110
        # a K step of 32 rows starting before n stays inside the panel column
        assert L.panel_ld >= 4000 + 32 and L.panel_ld % 128 == 0
        assert 1 <= L.split_k <= 16 and L.panel_elem_bytes == 4   # split-K from the tuned tile table
        assert L.total == ws
        offs = [L.omega, L.q_panel, L.compressed, L.evals, L.weights, L.factor, L.power_vec]
        assert all(o % 256 == 0 and o < ws for o in offs)
    finally:
        pp.psdproj_plan_destroy(plan)


def test_batch_workspace_covers_members():
    plans = [pp.psdproj_plan(n, 8, 4)[0] for n in (64, 500, 1333)]
    try:
        total = pp.psdproj_batch_workspace(plans)
        singles = [plan_status(n=n, k=8, p=4, q=0)[1] for n in (64, 500, 1333)]
        assert total >= max(singles)
    finally:
        for p in plans:
            pp.psdproj_plan_destroy(p)


def test_run_validates_before_touching_the_device():
    plan, ws = pp.psdproj_plan(100, 10, 5)
    try:
        fake = 1 << 20
        run = pp.lib.psdproj_run
        assert run(plan, None, 100, fake, 100, fake, fake, None) == pp.E_INVALID       # null A
        assert run(plan, fake, 99, fake * 4, 100, fake, fake, None) == pp.E_INVALID     # lda < n
        assert run(plan, fake + 4, 100, fake * 4, 100, fake, fake, None) == pp.E_INVALID  # misaligned A
        assert run(plan, fake, 100, fake * 4, 100, fake + 16, fake, None) == pp.E_INVALID  # misaligned workspace
        assert run(plan, fake, 100, fake + 400, 100, fake * 8, fake * 16, None) == pp.E_INVALID  # partial overlap
        assert run(None, fake, 100, fake, 100, fake, fake, None) == pp.E_INVALID
    finally:
        pp.psdproj_plan_destroy(plan)


def test_status_strings():
    for s in range(10):
        assert isinstance(pp.psdproj_status_str(s), str) and pp.psdproj_status_str(s)
    assert pp.psdproj_status_str(0) == "ok"


def test_server_create_without_device_fails_cleanly():
    """On a host without a GPU the server reports an error status instead of crashing."""
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import paper_2410_19208_amd as pp
    with pytest.raises(pp.PsdprojError):
        pp.psdproj_server_create(1 << 20, 4)
    with pytest.raises(pp.PsdprojError):
        pp.psdproj_server_create(16, 4)   # budget below the minimum: E_INVALID


def test_tile_table_is_used_by_the_planner():
    """Every entry of the tuner's table (csrc/tile_table.inc) is a valid split-K for its bucket,
    and a plan in that bucket takes the table's factor (after the planner's rounding of K chunks
    to whole 64-row steps); an override wins over the table and 0 restores it."""
    import re
    txt = open(os.path.join(ROOT, "paper_2410_19208_amd", "csrc", "tile_table.inc")).read()
    rows = [tuple(int(x) for x in m.groups()) for m in re.finditer(r"\{(-?\d+), (\d+), (\d+), (\d+)\}", txt)]
    rows = [r for r in rows if r[0] >= 0]
    assert rows, "tile table is empty"
    seen = set()
    for prec, b, rpad, split in rows:
        assert (prec, b, rpad) not in seen
        seen.add((prec, b, rpad))
        assert prec in (0, 1, 2) and 6 <= b <= 14 and rpad % 32 == 0 and 1 <= split <= 16
    for prec, b, rpad, split in rows[:: max(1, len(rows) // 25)]:
        n = 20000 if b == 14 else int(round(2 ** (b + 0.5)))
        k = rpad - 13
        if k < 1 or rpad - 3 > n:
            continue
        plan, _ = pp.psdproj_plan(n, k, 10, 0, pp.PLAIN, prec)
        try:
            L = pp.psdproj_plan_layout(plan)
            kchunk = -(-(-(-n // split)) // 64) * 64 if prec != 0 else None
            expect = -(-n // kchunk) if kchunk else split
            assert L.split_k == expect, (prec, b, rpad, split, L.split_k)
        finally:
            pp.psdproj_plan_destroy(plan)
    pp.psdproj_tile_override(pp.BF16X3, 3)
    try:
        plan, _ = pp.psdproj_plan(4096, 100, 10, 0, pp.PLAIN, pp.BF16X3)
        assert pp.psdproj_plan_layout(plan).split_k == 3
        pp.psdproj_plan_destroy(plan)
    finally:
        pp.psdproj_tile_override(pp.BF16X3, 0)
