"""The C-ABI library loads and exports every symbol include/pflbm.h declares;
host-side validation rejects invalid parameters (no GPU call is made)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2511_11360_amd import pflbm as P
from paper_2511_11360_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pflbm.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pflbm_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = P.lib()
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
        assert n in P.SIGNATURES, "binding lacks " + n


def test_struct_layout_matches_header(tmp_path):
    """ctypes structures have the C compiler's size and field offsets."""
    prog = ["#include <stdio.h>", "#include <stddef.h>", '#include "pflbm.h"', "int main(void){"]
    for S in (P.pflbm_params, P.pflbm_diag):
        prog.append('printf("%%zu\\n", sizeof(%s));' % S.__name__)
        for f, _ in S._fields_:
            prog.append('printf("%%zu\\n", offsetof(%s, %s));' % (S.__name__, f))
    prog.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(prog))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    exp = []
    for S in (P.pflbm_params, P.pflbm_diag):
        exp.append(ctypes.sizeof(S))
        exp.extend(getattr(S, f).offset for f, _ in S._fields_)
    assert got == exp


def _bytes(d, **kw):
    p = P.make_params(d, **kw)
    n = ctypes.c_size_t()
    st = P.lib().pflbm_state_bytes(ctypes.byref(p), ctypes.byref(n))
    return st, n.value


def test_state_bytes_sizes():
    d, _, _ = wl.static_droplet_2d()
    st, n = _bytes(d)
    assert st == 0
    # g 2 x 9 + h 2 x 5 populations of 4096 nodes in float64 (two buffers each)
    assert n >= (18 + 10) * 4096 * 8
    st, n16 = _bytes(d, precision="mixed_fp16")
    assert st == 0 and n16 < n
    d3 = wl.base_params(lattice="D3Q19_D3Q7", nx=32, ny=32, nz=32)
    st, n3 = _bytes(d3, precision="fp32")
    # AC on D3Q7 stores 6 phase-field populations per buffer
    assert st == 0 and n3 >= (38 + 12) * 32768 * 4


@pytest.mark.parametrize("bad", [
    dict(nu_H=0.0), dict(nu_L=-1.0), dict(W=0.0), dict(M=0.0), dict(sigma=-1.0),
    dict(rho_L=0.0), dict(s_other=2.0), dict(nx=0), dict(nz=2),
    dict(bc=("wall", "wall", "periodic")),
    dict(bc=("periodic", "wall", "periodic"), wall_u=((0.0, 0.1, 0.0), (0.0, 0.0, 0.0))),
    dict(gravity=(0.0, 0.0, 1e-5)),
    dict(normal_eps=-1.0),
])
def test_invalid_params_rejected(bad):
    d = wl.base_params(**bad)
    st, _ = _bytes(d)
    assert st == P.PFLBM_EINVAL


def test_d3q27_state_bytes_and_invalid_lattice():
    d = wl.base_params(lattice="D3Q27_D3Q7", nx=16, ny=16, nz=16)
    st, n = _bytes(d, precision="fp32")
    # g 2 x 27 and h 2 x 6 populations of 4096 nodes in float32
    assert st == 0 and n >= (54 + 12) * 4096 * 4
    p = P.make_params(d, "fp32")
    p.lattice = 3
    m = ctypes.c_size_t()
    assert P.lib().pflbm_state_bytes(ctypes.byref(p), ctypes.byref(m)) == P.PFLBM_EINVAL


def test_invalid_tile_rejected():
    d = wl.base_params(lattice="D3Q19_D3Q7", nx=32, ny=32, nz=32)
    for tile, ok in ((0, True), (3, True), (4, True), (5, True), (6, False), (-1, False)):
        p = P.make_params(d, "fp32", tile=tile)
        n = ctypes.c_size_t()
        st = P.lib().pflbm_state_bytes(ctypes.byref(p), ctypes.byref(n))
        assert (st == 0) == ok, tile


def test_size_limits():
    """Limits of the addressing: fewer than 2^31 nodes, and one z plane of a
    population (padded to 64 nodes) below 4 GiB, since kernels address it as a
    scalar base plus a 32-bit byte offset (float64: 2^29 nodes per plane)."""
    cases = [
        (dict(nx=23168, ny=23168), "fp64", True),      # 536 739 840 nodes, padded x 8 < 2^32
        (dict(nx=23171, ny=23171), "fp64", False),     # 536 895 241 x 8 > 2^32
        (dict(nx=32767, ny=32768), "fp32", True),      # 1 073 709 056 x 4 < 2^32
        (dict(nx=32768, ny=32768), "fp32", False),     # 2^30 x 4 = 2^32
        (dict(nx=32768, ny=32768), "mixed_fp16", False),
        (dict(lattice="D3Q19_D3Q7", nx=1290, ny=1290, nz=1290), "fp32", True),   # 2.147e9 < 2^31 nodes
        (dict(lattice="D3Q19_D3Q7", nx=1291, ny=1291, nz=1291), "fp32", False),  # over 2^31 - 1 nodes
    ]
    for kw, prec, ok in cases:
        st, _ = _bytes(wl.base_params(**kw), precision=prec)
        assert (st == 0) == ok, (kw, prec)


def test_strerror():
    L = P.lib()
    assert L.pflbm_strerror(P.PFLBM_EUNSTABLE).decode().startswith("numerical")
    assert L.pflbm_create(None, None, None, 0, None) == P.PFLBM_EINVAL


def test_every_handle_entry_point_rejects_a_null_handle():
    """Each entry point that takes a handle returns PFLBM_EINVAL for a null
    one (all other arguments null or zero too) before any HIP call, so this
    runs without a GPU; pflbm_last_error names the null handle."""
    import ctypes
    from paper_2511_11360_amd import pflbm as P
    L = P.lib()
    skip = {"pflbm_state_bytes", "pflbm_create", "pflbm_probe_bytes", "pflbm_probe_stream", "pflbm_destroy",
            "pflbm_last_error", "pflbm_strerror"}
    checked = 0
    for name, (res, args) in P.SIGNATURES.items():
        if name in skip:
            continue
        vals = [0 if a in (ctypes.c_int, ctypes.c_double, ctypes.c_size_t) else None for a in args]
        assert getattr(L, name)(*vals) == P.PFLBM_EINVAL, name
        checked += 1
    assert checked >= 28
    assert L.pflbm_last_error(None) == b"null handle"
    L.pflbm_destroy(None)   # a no-op


def test_create_rejects_small_or_misaligned_buffers_without_a_gpu():
    """pflbm_create checks the caller's buffer (null, fewer bytes than
    pflbm_state_bytes, not 256-byte aligned) before any HIP call."""
    import ctypes
    from paper_2511_11360_amd import pflbm as P
    L = P.lib()
    d = wl.base_params(lattice="D3Q19_D3Q7", nx=16, ny=8, nz=4)
    p = P.make_params(d, "fp64", 0, 0, "auto")
    nb = ctypes.c_size_t()
    assert L.pflbm_state_bytes(ctypes.byref(p), ctypes.byref(nb)) == 0
    h = ctypes.c_void_p()
    for ptr, size in ((None, nb.value), (4096, nb.value - 1), (4096 + 128, nb.value)):
        assert L.pflbm_create(ctypes.byref(p), None, ptr, size, ctypes.byref(h)) == P.PFLBM_EINVAL
        assert not h.value
    assert L.pflbm_create(None, None, 4096, nb.value, ctypes.byref(h)) == P.PFLBM_EINVAL
