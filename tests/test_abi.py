"""The C-ABI library loads and exports every symbol include/cgkmc.h declares (no GPU needed);
argument validation and arena sizing run on the host."""
import ctypes as C
import os
import re

import pytest

import paper_1407_5026_amd as cg
from workloads import headline, serial_small, uneven_batch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "cgkmc.h")).read()
    return sorted(set(re.findall(r"\b(cg_[a-z_A-Z]+)\s*\(", src)))


def test_header_declarations_match_binding():
    assert set(_declared()) == set(cg.EXPORTS)


def test_library_exports_every_symbol():
    lib = cg.load()
    for name in _declared():
        assert hasattr(lib, name), name


def test_struct_layouts_match_header(tmp_path):
    """ctypes mirrors of the ABI structs have the C compiler's sizes and field offsets."""
    import shutil
    import subprocess

    if not shutil.which("gcc"):
        pytest.skip("gcc unavailable")
    lines = []
    for st in (cg.cg_sample_desc, cg.cg_run_opts, cg.cg_stats):
        name = st.__name__
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in st._fields_:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "cgkmc.h"\nint main(void){'
                   + "".join(lines) + "return 0;}\n")
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                   check=True).stdout.splitlines())
    for st in (cg.cg_sample_desc, cg.cg_run_opts, cg.cg_stats):
        name = st.__name__
        assert int(got[name]) == C.sizeof(st), name
        for f, _ in st._fields_:
            assert int(got[f"{name}.{f}"]) == getattr(st, f).offset, (name, f)


def test_arena_bytes_and_validation():
    n = cg.arena_bytes(serial_small(), cg.make_opts())
    assert n > 0 and n % 256 == 0
    big = cg.arena_bytes(headline(256), cg.make_opts(precision=cg.CG_FP32_REFRESH))
    assert big > 256 * 16384 * 4
    cg.arena_bytes(uneven_batch(), cg.make_opts(precision=cg.CG_FP32_REFRESH))
    assert cg.arena_bytes([dict(serial_small()[0].as_dict(), M=16384)], cg.make_opts()) == n
    bad = dict(serial_small()[0].as_dict())
    for key, val in (("rc", 8.0), ("T", 0.0), ("L", 2), ("n_e", 0), ("xi", -1.0), ("M", 3), ("M", -2),
                     ("M", 1 << 25)):
        d = dict(bad)
        d[key] = val
        with pytest.raises(cg.CgError) as e:
            cg.arena_bytes([d], cg.make_opts())
        assert e.value.code == cg.CG_EINVAL
        assert cg.load().cg_last_error()
    for o in (cg.make_opts(block=300), cg.make_opts(M=1000), cg.make_opts(block=256),
              cg.make_opts(precision=7), cg.make_opts(clock_mode=5), cg.make_opts(phase_timers=3)):
        with pytest.raises(cg.CgError):
            cg.arena_bytes(serial_small(), o)


def test_pair_hop_configurations_refused_on_the_host():
    """Pair hops: square lattices, L <= 128, FP64 form, variant 0 or 1, 0 <= pair < 1."""
    from workloads import Sample

    ok = Sample(32, 512, 1.0, 1.0, 8.0, 0.06, 0.01, 48, 0, pair=0.2)
    assert cg.arena_bytes([ok], cg.make_opts(precision=cg.CG_FP64)) > 0
    bad = [
        ([ok], cg.make_opts(precision=cg.CG_FP32_REFRESH)),
        ([ok], cg.make_opts(precision=cg.CG_FP64, variant=5)),
        ([ok], cg.make_opts(precision=cg.CG_FP64, variant=6)),
        ([ok], cg.make_opts(precision=cg.CG_FP64, block=512)),
        ([Sample(256, 32768, 1.0, 1.0, 10.0, 0.05, 0.005, 1, 0, pair=0.1)], cg.make_opts(precision=cg.CG_FP64)),
        ([Sample(32, 512, 1.0, 1.0, 8.0, 0.06, 0.01, 48, 0, pair=1.0)], cg.make_opts(precision=cg.CG_FP64)),
        ([Sample(32, 512, 1.0, 1.0, 8.0, 0.06, 0.01, 48, 0, pair=-0.1)], cg.make_opts(precision=cg.CG_FP64)),
        ([Sample(8, 256, 1.0, 1.0, 2.0, 0.06, 0.01, 48, 0, dim=3, pair=0.1)], cg.make_opts(precision=cg.CG_FP64)),
    ]
    for samples, opts in bad:
        with pytest.raises(cg.CgError) as e:
            cg.arena_bytes(samples, opts)
        assert e.value.code == cg.CG_EINVAL
