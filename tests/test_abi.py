"""CPU checks of the boundary: the C-ABI library loads and exports every
declared entry point, argument validation fails cleanly before any device
call, and the product and the oracle stay independent."""
import ast
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ib[o]?_[a-z0-9_]+)\s*\(", text)))


def _lib():
    from paper_math_0301321_amd import ib
    return ib.load_library()


def test_library_exports_every_declared_entry_point():
    lib = _lib()
    names = _declared(os.path.join(ROOT, "include", "ib.h"))
    assert "ib_step" in names and "ib_adjoint_step" in names
    for name in names:
        assert hasattr(lib, name), name


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes structures have the field offsets and sizes that a C
    compiler gives the structures of include/ib.h."""
    import subprocess
    from paper_math_0301321_amd import ib
    structs = {"ib_params": ib.ib_params, "ib_lattice": ib.ib_lattice, "ib_elastic": ib.ib_elastic}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ib.h"', "int main(void) {"]
    for sname, cls in structs.items():
        lines.append(f'  printf("{sname} size %zu\\n", sizeof({sname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{sname} {fname} %zu\\n", offsetof({sname}, {fname}));')
    lines.append("  return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for sname, cls in structs.items():
        assert got[(sname, "size")] == C.sizeof(cls), sname
        for fname, _ in cls._fields_:
            assert got[(sname, fname)] == getattr(cls, fname).offset, (sname, fname)


def test_oracle_exports_every_declared_function(oracle_mod):
    lib = oracle_mod.lib()
    for name in _declared(os.path.join(ROOT, "oracle", "ibo.h")):
        assert hasattr(lib, name), name


def _params(ib, **kw):
    p = dict(n=16, L=1.0, rho=1.0, mu=0.01, dt=1e-3, fluid_precision=ib.IB_FLUID_FP32, convect=1,
             n_markers=0, stream=None)
    p.update(kw)
    return ib.ib_params(**p)


@pytest.mark.parametrize("kw,code", [
    (dict(n=12), "IB_ENOTSUP"), (dict(n=4), "IB_ENOTSUP"), (dict(n=1024), "IB_ENOTSUP"),
    (dict(L=0.0), "IB_EINVAL"), (dict(rho=-1.0), "IB_EINVAL"), (dict(mu=-0.1), "IB_EINVAL"),
    (dict(dt=0.0), "IB_EINVAL"), (dict(dt=float("nan")), "IB_EINVAL"),
    (dict(fluid_precision=7), "IB_EINVAL"), (dict(convect=2), "IB_EINVAL"),
    (dict(n_markers=-5), "IB_EINVAL"), (dict(n_markers=10), "IB_EINVAL"),   # no material arrays
    (dict(n=16, nz=8), "IB_ENOTSUP"), (dict(n=512, nz=256), "IB_ENOTSUP"),  # half-cube needs n in 32..256
    (dict(n=64, nz=16), "IB_ENOTSUP"), (dict(n=64, nz=128), "IB_ENOTSUP"), (dict(n=64, nz=40), "IB_ENOTSUP"),
    (dict(n=16, nz=12), "IB_ENOTSUP"), (dict(n=512, nz=384), "IB_ENOTSUP"),   # 3n/4 needs n in 32..256
    (dict(displacement=2), "IB_EINVAL"), (dict(displacement=-1), "IB_EINVAL"),
])
def test_create_rejects_bad_parameters(kw, code):
    from paper_math_0301321_amd import ib
    lib = _lib()
    p = _params(ib, **kw)
    e = ib.ib_elastic()
    h = C.c_void_p()
    rc = lib.ib_create(C.byref(p), C.byref(e), C.byref(h))
    assert rc == getattr(ib, code)
    assert h.value is None
    assert lib.ib_last_error(None).decode().startswith("ib_create")


def test_create_rejects_bad_topology():
    from paper_math_0301321_amd import ib
    lib = _lib()
    fake = C.c_void_p(16)     # never dereferenced: validation fails first
    p = _params(ib, n_markers=10)
    lat = (ib.ib_lattice * 1)(ib.ib_lattice(0, 4, 3, 0, 1.0, 0.0))          # 12 > 10 markers
    e = ib.ib_elastic(w=fake, k=fake, X_ref=fake, n_lattices=1, lattices=lat)
    assert lib.ib_create(C.byref(p), C.byref(e), C.byref(C.c_void_p())) == ib.IB_EINVAL
    lat = (ib.ib_lattice * 1)(ib.ib_lattice(0, 5, 2, 1, 1.0, 0.0))          # periodic with n2 < 3
    e = ib.ib_elastic(w=fake, k=fake, X_ref=fake, n_lattices=1, lattices=lat)
    assert lib.ib_create(C.byref(p), C.byref(e), C.byref(C.c_void_p())) == ib.IB_EINVAL
    ab = np.array([[0, 3], [3, 3]], np.int32)                               # spring (3, 3)
    rest = np.array([0.1, 0.1])
    e = ib.ib_elastic(w=fake, k=fake, X_ref=fake, n_springs=2, spring_ab=ab.ctypes.data_as(C.c_void_p),
                      spring_rest=rest.ctypes.data_as(C.c_void_p))
    assert lib.ib_create(C.byref(p), C.byref(e), C.byref(C.c_void_p())) == ib.IB_EINVAL
    di = np.array([1, 1], np.int32)                                         # repeated drive index
    dd = np.zeros((3, 2))
    e = ib.ib_elastic(w=fake, k=fake, X_ref=fake, n_drive=2, drive_idx=di.ctypes.data_as(C.c_void_p),
                      drive_dir=dd.ctypes.data_as(C.c_void_p))
    assert lib.ib_create(C.byref(p), C.byref(e), C.byref(C.c_void_p())) == ib.IB_EINVAL


def test_null_context_calls_fail_cleanly():
    from paper_math_0301321_amd import ib
    lib = _lib()
    assert lib.ib_step(None, None, None, 0.0, None) == ib.IB_EINVAL
    assert lib.ib_adjoint_step(None, None, None, 0.0, None, None, None) == ib.IB_EINVAL
    assert lib.ib_bin_reuse(None, 1) == ib.IB_EINVAL
    assert lib.ib_workspace_bytes(None) == 0


def test_fluid_noalloc_validates_before_any_device_call():
    """Sizes beyond the static scratch and bad parameters are refused with a
    clear error before the entry point touches a device."""
    from paper_math_0301321_amd import ib
    lib = _lib()
    fake = C.c_void_p(0x1000)       # never dereferenced: validation fails first

    def params(n, nz=0, prec=ib.IB_FLUID_FP32, **kw):
        d = dict(L=1.0, rho=1.0, mu=0.01, dt=1e-3, convect=1)
        d.update(kw)
        return ib.ib_params(n, d["L"], d["rho"], d["mu"], d["dt"], prec, d["convect"], 0, None, nz)

    assert lib.ib_fluid_noalloc(None, fake, None) == ib.IB_EINVAL
    assert lib.ib_fluid_noalloc(C.byref(params(64)), None, None) == ib.IB_EINVAL
    for n, nz in ((48, 0), (16, 0), (512, 0), (64, 16)):
        assert lib.ib_fluid_noalloc(C.byref(params(n, nz)), fake, None) == ib.IB_ENOTSUP, (n, nz)
    for kw in (dict(rho=0.0), dict(dt=-1.0), dict(mu=-1.0), dict(convect=2), dict(L=float("nan"))):
        assert lib.ib_fluid_noalloc(C.byref(params(64, **kw)), fake, None) == ib.IB_EINVAL, kw
    # beyond 32 MiB: 256^3 in FP32 (203 MB of spectrum), 128^3 in FP64 (51 MB)
    for n, nz, prec in ((256, 0, ib.IB_FLUID_FP32), (256, 128, ib.IB_FLUID_FP32), (128, 0, ib.IB_FLUID_FP64)):
        assert lib.ib_fluid_noalloc(C.byref(params(n, nz, prec)), fake, None) == ib.IB_ENOTSUP, (n, nz, prec)
        msg = lib.ib_last_error(None).decode()
        assert "limit is 33554432" in msg, msg


def _imports(path):
    tree = ast.parse(open(path).read())
    out = set()
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            out |= {a.name.split(".")[0] for a in node.names}
        elif isinstance(node, ast.ImportFrom) and node.module:
            out.add(node.module.split(".")[0])
    return out


def test_product_and_oracle_are_independent():
    pkg = os.path.join(ROOT, "paper_math_0301321_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith(".py"):
                assert "oracle" not in _imports(os.path.join(dirpath, f)), f
            if f.endswith((".hip", ".h", ".cpp")):
                assert "ibo" not in open(os.path.join(dirpath, f)).read(), f
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith(".py"):
            assert "paper_math_0301321_amd" not in _imports(os.path.join(ROOT, "oracle", f)), f
        if f.endswith((".c", ".h")):
            txt = open(os.path.join(ROOT, "oracle", f)).read()
            assert "ib_internal" not in txt and "include/ib.h" not in txt, f


def test_bench_byte_model_covers_every_timed_kernel():
    """bench.py prices every single-kernel phase it may pick as the roofline kernel."""
    import importlib.util
    import os
    spec = importlib.util.spec_from_file_location("bench", os.path.join(os.path.dirname(__file__), "..", "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    from paper_math_0301321_amd import workloads as W
    wl = W.tiny_helix()
    wls = bench.worklist_sizes(wl)
    assert wls["items"] >= wls["tiles_with_markers"] > 0 and wls["tiles_touched"] >= wls["tiles_with_markers"]
    for phase, kernel in bench.SINGLE_KERNEL.items():
        v = bench.phase_bytes(phase, wl.N, wl.M, 4, wls)
        assert v is not None and (v > 0 or (phase == "split" and wls["split_tiles"] == 0)), phase
        assert kernel in bench.KERNEL_SOURCE


def test_bench_byte_model_on_the_half_cube():
    """The byte model and work-list sizes on an n x n x n/2 grid: the grid and
    spectrum terms are half the cube's, and the binning sees the tiles of the
    half-height box."""
    import importlib.util
    import os
    spec = importlib.util.spec_from_file_location("bench", os.path.join(os.path.dirname(__file__), "..", "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    from paper_math_0301321_amd import workloads as W
    wl = W.tiny_halfcube(32)
    wls = bench.worklist_sizes(wl)
    assert wls["tiles_touched"] <= (32 // 8) ** 2 * (16 // 8)
    n, nz, b = 32, 16, 4
    G, spec_b = n * n * nz, 3 * (n // 2 + 1) * n * nz * 2 * b
    assert bench.phase_bytes("fft_y", n, wl.M, b, wls, nz) == 2 * spec_b
    assert bench.phase_bytes("fft_x_inv", n, wl.M, b, wls, nz) == spec_b + 3 * G * b
    assert bench.phase_bytes("fft_x_inv", n, wl.M, b, wls, nz) * 2 == bench.phase_bytes("fft_x_inv", n, wl.M, b, wls)
