"""Host-side checks of the C ABI: the library loads, exports every declared
entry point, validates arguments before touching a device, and plans the
phase schedule and tile geometry the paper's structural numbers imply.
No test here launches a kernel."""
import ctypes
import os
import re

import pytest

import paper_1612_02495_amd as P
from paper_1612_02495_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "swept.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    names = _declared_functions()
    assert len(names) >= 9
    lib = _lib.lib()
    for n in names:
        assert hasattr(lib, n), n


def test_header_declares_the_boundary():
    names = set(_declared_functions())
    for n in ("swept_plan_create", "swept_run", "naive_run", "swept_plan_info", "swept_plan_destroy",
              "swept_last_error"):
        assert n in names


def test_header_is_plain_c(tmp_path):
    # the boundary takes plain pointers and sizes: the header compiles as
    # C99 with no warnings, and a C program can call every entry point
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "use.c"
    calls = "\n".join(f"  (void)&{n};" for n in _declared_functions())
    src.write_text(f'#include "swept.h"\nint main(void) {{\n{calls}\n  return 0;\n}}\n')
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I", os.path.dirname(HEADER),
                        "-fsyntax-only", str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def _create(n=1024, kind=0, dtype=1, dt=1e-6, dx=1e-3, alpha=1.0, w=64, spc=0):
    h = ctypes.c_void_p()
    rc = _lib.lib().swept_plan_create(ctypes.byref(h), n, kind, dtype, dt, dx, alpha, w, spc)
    return rc, h


@pytest.mark.parametrize("kw,code", [
    (dict(kind=7), _lib.SWEPT_EINVAL),
    (dict(dtype=3), _lib.SWEPT_EINVAL),
    (dict(n=2), _lib.SWEPT_EINVAL),
    (dict(dx=0.0), _lib.SWEPT_EINVAL),
    (dict(dt=float("nan")), _lib.SWEPT_EINVAL),
    (dict(alpha=float("inf")), _lib.SWEPT_EINVAL),
    (dict(w=-8), _lib.SWEPT_EINVAL),
    (dict(w=6, kind=1), _lib.SWEPT_EINVAL),     # KS: multiple of 8
    (dict(w=3), _lib.SWEPT_EINVAL),             # heat: below minimum / odd
    (dict(w=8192), _lib.SWEPT_EINVAL),
    (dict(w=96), _lib.SWEPT_EUNSUPPORTED),      # 1024 % 96 != 0
    (dict(n=31, w=0), _lib.SWEPT_EUNSUPPORTED),    # odd n below the uneven tiling: no tile width
    (dict(n=1023, w=256), _lib.SWEPT_EUNSUPPORTED),  # uneven tiles need width 512 or 1024
    (dict(n=1023, w=512, kind=2), _lib.SWEPT_EUNSUPPORTED),  # not for the insulated rod
    (dict(spc=33), _lib.SWEPT_EINVAL),          # heat w=64: at most 32 steps per phase
    (dict(kind=1, w=64, spc=9), _lib.SWEPT_EINVAL),  # KS w=64: at most 8 steps per phase
    (dict(kind=3), _lib.SWEPT_EINVAL),
    (dict(kind=2, w=64), _lib.SWEPT_EUNSUPPORTED),   # insulated rod: tile_width 512 or 1024 only
    (dict(kind=2, alpha=float("nan")), _lib.SWEPT_EINVAL),
])
def test_plan_create_rejects_before_any_device_call(kw, code):
    rc, h = _create(**kw)
    assert rc == code
    assert not h.value
    assert P.swept_last_error()


def test_null_plan_entry_points():
    lib = _lib.lib()
    assert lib.swept_run(None, None, 1, None) == _lib.SWEPT_EINVAL
    assert lib.naive_run(None, None, 1, None) == _lib.SWEPT_EINVAL
    assert lib.swept_plan_info(None, None, None, None) == _lib.SWEPT_EINVAL
    assert lib.swept_plan_set_engine(None, 0) == _lib.SWEPT_EINVAL
    lib.swept_plan_destroy(None)
    assert lib.swept_plan_create(None, 1024, 0, 1, 1e-6, 1e-3, 1.0, 64, 0) == _lib.SWEPT_EINVAL
    with pytest.raises(P.SweptError):
        P.swept_plan_create(1024, "heat", "f64", 1e-6, 1e-3, 1.0, tile_width=100)


@pytest.mark.parametrize("kind,w,spc,steps,want", [
    ("heat", 64, 0, 1000, [32] * 31 + [8]),            # 1000 = 31 x 32 + 8
    ("heat", 1024, 0, 100000, [512] * 195 + [160]),    # 10^5 = 195 x 512 + 160
    ("ks", 1024, 0, 20000, [256] * 156 + [64]),        # 2 x 10^4 steps = 156 x 128 + 32
    ("heat", 64, 5, 12, [5, 5, 2]),
    ("ks", 64, 3, 7, [6, 6, 2]),
    ("heat", 16, 0, 0, []),
    ("heat", 16, 0, 3, [3]),
])
def test_schedule(kind, w, spc, steps, want):
    got = P.swept_schedule(kind, w, spc, steps)
    assert got == want
    tps = 2 if kind == "ks" else 1
    assert sum(got) == steps * tps
    if kind == "ks":
        assert all(h % 2 == 0 for h in got)


def test_schedule_rejects_bad_arguments():
    lib = _lib.lib()
    cnt = ctypes.c_int64()
    assert lib.swept_schedule(0, 64, 0, -1, None, 0, ctypes.byref(cnt)) == _lib.SWEPT_EINVAL
    assert lib.swept_schedule(0, 63, 0, 10, None, 0, ctypes.byref(cnt)) == _lib.SWEPT_EINVAL
    assert lib.swept_schedule(0, 64, 0, 10, None, 5, ctypes.byref(cnt)) == _lib.SWEPT_EINVAL
    assert lib.swept_schedule(0, 64, 0, 10, None, 0, None) == _lib.SWEPT_EINVAL


def _golden():
    out = {}
    for line in open(os.path.join(ROOT, "tests", "golden", "paper_tiling.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            key, val, _cite = line.split()
            out[key] = int(val)
    return out


def test_paper_tiling_numbers():
    g = _golden()
    # Sec. 4.2: one full triangle of a 512-point node holds 65792 values,
    # i.e. tiers of 512, 510, ..., 2 values.
    geo = P.swept_tile_geometry("heat", 512)
    tiers = geo["full_tiers"]
    assert sum(512 - 2 * k for k in range(tiers)) == g["triangle_values_w512_heat"]
    # Sec. 4.2: the two-row matrix holds 2 (n + 2) values.
    assert 2 * geo["row_values"] == g["two_row_values_w512_heat"]
    # Sec. 6: a 32-point KS node advances 4 timesteps per cycle.
    ks = P.swept_tile_geometry("ks", 32)
    assert ks["full_tiers"] // 2 == g["ks_steps_per_cycle_w32"]
    assert P.swept_schedule("ks", 32, 0, 4) == [8]


def test_edge_slot_geometry():
    for kind, s in (("heat", 1), ("ks", 2)):
        for w in (8, 64, 1024):
            geo = P.swept_tile_geometry(kind, w)
            assert geo["edge_slot_values"] == 2 * (w // 2 + s)
            assert geo["row_values"] == w + 2 * s


def test_insulated_rod_shares_the_heat_tiling():
    # the insulated rod runs the heat stencil on the same ring of tiles
    for w in (512, 1024):
        assert P.swept_tile_geometry("heat_insulated", w) == P.swept_tile_geometry("heat", w)
        assert P.swept_schedule("heat_insulated", w, 0, 1000) == P.swept_schedule("heat", w, 0, 1000)


def _noalloc(n=1024, kind=0, dtype=1, dt=1e-6, dx=1e-3, alpha=1.0, w=64, spc=0, u=1, steps=10):
    return _lib.lib().swept_run_noalloc(n, kind, dtype, dt, dx, alpha, w, spc, ctypes.c_void_p(u), steps, None)


@pytest.mark.parametrize("kw,code", [
    (dict(kind=7), _lib.SWEPT_EINVAL),
    (dict(dx=0.0), _lib.SWEPT_EINVAL),
    (dict(w=96), _lib.SWEPT_EUNSUPPORTED),
    (dict(steps=-1), _lib.SWEPT_EINVAL),
    (dict(u=0), _lib.SWEPT_EINVAL),
    # edge slots beyond the 32 MiB static array: 2 (2^22 / 1024) 1026 x 8 bytes
    (dict(n=1 << 22, w=1024), _lib.SWEPT_EUNSUPPORTED),
    (dict(n=1 << 22, w=1024, kind=1), _lib.SWEPT_EUNSUPPORTED),
])
def test_noalloc_rejects_before_any_device_call(kw, code):
    # the pointer given for u is never dereferenced: every case fails first
    assert _noalloc(**kw) == code
    assert P.swept_last_error()


def test_noalloc_size_limit_message():
    assert _noalloc(n=1 << 22, w=1024) == _lib.SWEPT_EUNSUPPORTED
    msg = P.swept_last_error()
    assert "static workspace" in msg and str(2 * 4096 * 1026 * 8) in msg


def test_check_flags_validated_before_any_device_call():
    lib = _lib.lib()
    assert lib.swept_plan_set_checks(None, _lib.SWEPT_CHECK_NONFINITE) == _lib.SWEPT_EINVAL
    assert lib.swept_batch_set_checks(None, _lib.SWEPT_CHECK_NONFINITE) == _lib.SWEPT_EINVAL
    assert _lib.SWEPT_ENONFINITE == -5


def test_header_documents_status_codes():
    text = open(HEADER).read()
    for name, code in (("SWEPT_OK", 0), ("SWEPT_EINVAL", -1), ("SWEPT_EUNSUPPORTED", -2), ("SWEPT_ENOMEM", -3),
                       ("SWEPT_EDEVICE", -4), ("SWEPT_ENONFINITE", -5)):
        assert re.search(rf"#define {name} {code}\b", text), name
    assert "no time-out status" in text
