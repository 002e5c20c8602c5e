"""The C-ABI library on the CPU: it loads, exports every entry point that
include/ah.h declares, and rejects invalid problems before touching a GPU."""
import ctypes as C
import os
import re
import subprocess

import pytest

import paper_1809_00995_amd as AH
from paper_1809_00995_amd import ah as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ah.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ah_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_entry_point():
    lib = AH.load_library()
    names = declared_functions()
    assert len(names) == 13
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(B.EXPORTED) == names


def test_struct_layouts_match_the_header(tmp_path):
    """ctypes mirrors of ah_params, ah_buffers and ah_obs: every field offset
    and the total size equal what a C compiler makes of include/ah.h."""
    structs = {"ah_params": B._Params, "ah_buffers": B._Buffers, "ah_obs": B._Obs}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ah.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    for line in filter(None, out):
        cname, f, v = line.split()
        py = structs[cname]
        got = C.sizeof(py) if f == "size" else getattr(py, f).offset
        assert got == int(v), (cname, f)


def _init(**kw):
    lib = AH.load_library()
    p = AH.Params(64, 8, 8, **kw)._c()
    b = B._Buffers(4096)                      # never dereferenced: validation fails first
    ctx = C.c_void_p()
    rc = lib.ah_init(C.byref(ctx), 1, C.byref(p), C.byref(b), None)
    return rc, lib.ah_last_error(None).decode(), ctx


@pytest.mark.parametrize("kw,code,text", [
    (dict(dt=0.3), B.AH_E_DOMAIN, "CFL"),
    (dict(s=1.5), B.AH_E_DOMAIN, "s must"),
    (dict(s=-5.0), B.AH_E_DOMAIN, "s must"),
    (dict(s=-1.0, tau0=0.0), B.AH_E_DOMAIN, "s < 0"),
    (dict(tau_s=2.0, s_late=3.0), B.AH_E_DOMAIN, "s_late"),
    (dict(era_p=-1.0), B.AH_E_DOMAIN, "era_p"),
    (dict(tau_ref=0.0), B.AH_E_DOMAIN, "tau_ref"),
    (dict(tau0=-5.0), B.AH_E_DOMAIN, "a(tau"),
    (dict(init=7), B.AH_E_INVALID, "init"),
    (dict(n_end=-2), B.AH_E_INVALID, "n_end"),
    (dict(layout=2), B.AH_E_INVALID, "layout"),
])
def test_invalid_parameters_are_rejected(kw, code, text):
    rc, msg, ctx = _init(**kw)
    assert rc == code and text in msg and not ctx.value


def test_bad_extents_alignment_and_null():
    lib = AH.load_library()
    ctx = C.c_void_p()
    p = AH.Params(2, 8, 8)._c()
    b = B._Buffers(4096)
    assert lib.ah_init(C.byref(ctx), 1, C.byref(p), C.byref(b), None) == B.AH_E_INVALID
    p = AH.Params(64, 8, 8)._c()
    b = B._Buffers(4096 + 16)
    assert lib.ah_init(C.byref(ctx), 1, C.byref(p), C.byref(b), None) == B.AH_E_INVALID
    assert "aligned" in lib.ah_last_error(None).decode()
    assert lib.ah_init(C.byref(ctx), 0, C.byref(p), C.byref(b), None) == B.AH_E_INVALID
    assert lib.ah_init(None, 1, C.byref(p), C.byref(b), None) == B.AH_E_INVALID
    mixed = (B._Params * 2)(AH.Params(64, 8, 8)._c(), AH.Params(64, 8, 8, precision=1)._c())
    bufs = (B._Buffers * 2)(B._Buffers(4096), B._Buffers(8192))
    assert lib.ah_init(C.byref(ctx), 2, mixed, bufs, None) == B.AH_E_INVALID
    mixed = (B._Params * 2)(AH.Params(64, 8, 8, layout=0)._c(), AH.Params(64, 8, 8, layout=1)._c())
    assert lib.ah_init(C.byref(ctx), 2, mixed, bufs, None) == B.AH_E_INVALID
    assert "one layout" in lib.ah_last_error(None).decode()
    assert lib.ah_step(None, 1, 0, None, 0, None) == B.AH_E_INVALID
    assert lib.ah_free(None) == B.AH_OK
    assert lib.ah_error_string(B.AH_E_NONFINITE) == b"non-finite field values"


def test_noalloc_measure_rejects_bad_sizes_before_device_work():
    """ah_measure_noalloc holds at most AH_NOALLOC_MAX_REAL states in its static
    scratch: other counts and NULL arguments fail before any GPU call."""
    hdr = open(os.path.join(ROOT, "include", "ah.h")).read()
    assert int(re.search(r"#define AH_NOALLOC_MAX_REAL (\d+)", hdr).group(1)) == \
        B.AH_NOALLOC_MAX_REAL
    lib = AH.load_library()
    n = B.AH_NOALLOC_MAX_REAL + 1
    ps = (B._Params * n)(*[AH.Params(64, 8, 8)._c() for _ in range(n)])
    bs = (B._Buffers * n)(*[B._Buffers(4096) for _ in range(n)])
    assert lib.ah_measure_noalloc(n, ps, bs, 4096, None, None) == B.AH_E_INVALID
    msg = lib.ah_last_error(None).decode()
    assert "static scratch" in msg and str(B.AH_NOALLOC_MAX_REAL) in msg
    assert lib.ah_measure_noalloc(0, ps, bs, 4096, None, None) == B.AH_E_INVALID
    assert lib.ah_measure_noalloc(1, ps, bs, None, None, None) == B.AH_E_INVALID
    assert lib.ah_measure_noalloc(1, None, bs, 4096, None, None) == B.AH_E_INVALID
    bad = (B._Params * 1)(AH.Params(64, 8, 8, dt=0.3)._c())
    assert lib.ah_measure_noalloc(1, bad, bs, 4096, None, None) == B.AH_E_DOMAIN


def test_slab_parameters_are_validated():
    """z_halo (a z-slab of a larger lattice) must be 0, 1 or 2 with reserved 0, shared by
    every realization, and a slab needs nx % 64 == 0 and AH_INIT_NONE or AH_INIT_VACUUM;
    all refused before any device work."""
    lib = AH.load_library()
    ctx = C.c_void_p()
    b = B._Buffers(4096)
    none = dict(init=AH.AH_INIT_NONE)

    def init(*ps):
        arr = (B._Params * len(ps))(*[q._c() for q in ps])
        bufs = (B._Buffers * len(ps))(*[B._Buffers(4096 * (k + 1)) for k in range(len(ps))])
        return lib.ah_init(C.byref(ctx), len(ps), arr, bufs, None)

    assert init(AH.Params(64, 8, 8, z_halo=3, **none)) == B.AH_E_INVALID
    assert "z_halo" in lib.ah_last_error(None).decode()
    assert init(AH.Params(64, 8, 8, z_halo=-1, **none)) == B.AH_E_INVALID
    bad = AH.Params(64, 8, 8, z_halo=2, **none)._c()
    bad.reserved = 1
    assert lib.ah_init(C.byref(ctx), 1, C.byref(bad), C.byref(b), None) == B.AH_E_INVALID
    assert init(AH.Params(32, 8, 8, z_halo=2, **none)) == B.AH_E_INVALID
    assert "nx % 64" in lib.ah_last_error(None).decode()
    assert init(AH.Params(64, 8, 8, z_halo=2)) == B.AH_E_INVALID   # random-phase start
    assert "AH_INIT_NONE" in lib.ah_last_error(None).decode()
    assert init(AH.Params(64, 8, 8, z_halo=2, **none), AH.Params(64, 8, 8, **none)) == \
        B.AH_E_INVALID
    assert "one z_halo" in lib.ah_last_error(None).decode()
    # stored sites include the halo planes
    q = AH.Params(64, 8, 8, z_halo=2)
    assert q.nz_stored == 12 and q.sites == 64 * 8 * 12


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; --gpus N > 1 exits with a message before touching a GPU."""
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    res = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr and res.stdout == ""


def test_observation_records_decode_like_field_by_field_reads():
    """ObsRecords.decode (one NumPy pass over the ah_obs array) gives the Obs a
    field-by-field ctypes read gives, for every field kind: integers, doubles,
    NaN, and the fixed-size arrays."""
    n_slots, n_real = 3, 5
    out = (B._Obs * (n_slots * n_real))()
    for k in range(n_slots * n_real):
        o = out[k]
        o.step, o.tau, o.a, o.n_wind = 20 * k, 0.1 * k + 1.0, 2.0 ** -k, 7 * k - 3
        o.n_wind_dir[2], o.net_wind_dir[0], o.nonfinite = k, -k, k % 2
        o.v2[1], o.num[0], o.den[2] = 0.25 * k, -1e300, 3e-310
        o.xi_l = float("nan") if k % 3 == 0 else 1.5 * k
        o.energy, o.pres_lag, o.v2_eos = -0.5 * k, 1e-17 * k, 0.3
    rec = B.ObsRecords(out, n_slots, n_real)
    got = rec.decode()
    assert len(rec) == n_slots and [len(s) for s in got] == [n_real] * n_slots
    for j in range(n_slots):
        for r in range(n_real):
            ref = B.Obs._from(out[j * n_real + r])
            g = got[j][r]
            for name in B.Obs.__dataclass_fields__:
                a, b = getattr(g, name), getattr(ref, name)
                assert type(a) is type(b), name
                if isinstance(b, float) and b != b:
                    assert a != a, name
                else:
                    assert a == b, name


def test_bench_secondary_form_failure_keeps_the_line():
    """A secondary form of bench.py that fails (an exception, or run_form's exit when too
    few steps are given) records its error in its own entry; the forms after it and the
    headline line are still produced."""
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench

    def boom():
        raise RuntimeError("out of memory")

    def too_few():
        raise SystemExit("bench.py: no unmeasured 2-step call to time the kernel by")

    line = {}
    bench.secondary(line, "a", boom)
    bench.secondary(line, "b", too_few)
    bench.secondary(line, "c", lambda: {"value": 1.0})
    assert line["a"] == {"error": "RuntimeError: out of memory"}
    assert line["b"]["error"].startswith("SystemExit: bench.py: no unmeasured")
    assert line["c"] == {"value": 1.0}
