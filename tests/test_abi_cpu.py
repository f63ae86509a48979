"""Host-side checks of the C ABI that need no GPU: the in-tree library loads,
exports every symbol declared in include/pflbm.h, sizes workspaces and
rejects invalid parameters."""
import os
import re

import pytest

from paper_2207_09431_amd import inputs, pflbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "pflbm.h")).read()
    return sorted(set(re.findall(r"\b(pflbm_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(pflbm.LIB_PATH):
        pytest.fail("libpflbm.so is not built (run __graft_entry__.build())")
    return pflbm.lib()


def test_every_declared_symbol_is_exported(L):
    syms = declared_symbols()
    assert len(syms) >= 17
    assert set(syms) == set(pflbm.EXPORTS)
    for s in syms:
        assert hasattr(L, s), s


def test_workspace_bytes_valid_and_invalid(L):
    prm = inputs.rising_bubble_small()["params"]
    n = pflbm.workspace_bytes([prm])
    assert n > 9 * 2 * 4 * 64 * 128
    bad = [dict(prm, nx=4), dict(prm, n_h=3), dict(prm, rho=[0.0, 1.0, 1.0]), dict(prm, nu_min=2.0, nu_max=1.0,
           powerlaw_comp=2), dict(prm, tau_h=0.7, store_h=0), dict(prm, sigma23=1.0), dict(prm, xi=0.0),
           dict(prm, tau_iterations=-1), dict(prm, tau_iterations=9),
           dict(prm, powerlaw_comp=2, n=0.0), dict(prm, powerlaw_comp=2, K=float("inf")),
           dict(prm, xi=float("inf")), dict(prm, D0=float("nan")), dict(prm, tau_h=float("inf"), store_h=1),
           dict(prm, hforce_cd=2), dict(prm, open_x=2), dict(prm, open_x=1, u_in=float("nan")),
           dict(prm, mobility_flux=2)]
    for b in bad:
        assert pflbm.workspace_bytes([b]) == 0, b
    assert pflbm.workspace_bytes([dict(prm, tau_iterations=8)]) == n
    # a stored-hbar case with tau_h != 1/2 is valid
    assert pflbm.workspace_bytes([dict(prm, tau_h=0.7, store_h=1)]) > n
    # batched cases must agree on n_h / storage / store_h
    assert pflbm.workspace_bytes([prm, dict(prm, n_h=2)]) == 0
    assert pflbm.workspace_bytes([prm, dict(prm, nx=80, ny=90)]) > n
    assert pflbm.workspace_bytes([prm, dict(prm, storage=1)]) == 0
    assert pflbm.workspace_bytes([dict(prm, storage=2)]) == 0
    # the largest domain: pitch x ny just below 2^29 nodes (float64 planes under 4 GiB)
    assert pflbm.workspace_bytes([dict(prm, nx=16384, ny=32767)]) > 0
    assert pflbm.workspace_bytes([dict(prm, nx=16384, ny=32768)]) == 0
    assert pflbm.workspace_bytes([dict(prm, nx=16321, ny=32768)]) == 0   # pitch rounds up to 16384


def test_float16_form_is_smaller(L):
    prm = inputs.many_bubbles_crop()["params"]
    n32 = pflbm.workspace_bytes([prm])
    n16 = pflbm.workspace_bytes([dict(prm, storage=1)])
    plane = 256 * 512
    # per ping-pong buffer: 8 float32 deviation planes become 2 float32
    # momentum planes + 6 float16 pair-moment planes
    assert n32 - n16 == 2 * (8 * 4 - 2 * 4 - 6 * 2) * plane


def test_status_strings(L):
    for s in (0, -1, -2, -3, -4, -5, -6):
        assert L.pflbm_status_string(s)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built library every call raises: there is no fallback."""
    monkeypatch.setattr(pflbm, "_lib", None)
    monkeypatch.setattr(pflbm, "LIB_PATH", str(tmp_path / "libpflbm.so"))
    prm = inputs.rising_bubble_small()["params"]
    with pytest.raises(RuntimeError, match="missing"):
        pflbm.workspace_bytes([prm])
    with pytest.raises(RuntimeError, match="missing"):
        pflbm.Solver(prm)


def test_params_layout_matches_the_header(tmp_path):
    """The binding's ctypes mirror of pflbm_params has the header's size and
    every field at the header's offset (a C program compiled against
    include/pflbm.h prints them)."""
    import ctypes as ct
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    names = [f for f, _ in pflbm.Params._fields_]
    src = tmp_path / "layout.c"
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"pflbm.h\"\nint main(void) {\n"
                   "  printf(\"%zu\\n\", sizeof(pflbm_params));\n"
                   + "".join(f"  printf(\"%zu\\n\", offsetof(pflbm_params, {n}));\n" for n in names)
                   + "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert out[0] == ct.sizeof(pflbm.Params)
    assert out[1:] == [getattr(pflbm.Params, n).offset for n in names]


def test_set_state_rejects_host_and_non_byte_tensors():
    """The state copy is device to device: a host tensor, or one of another
    dtype, is refused before any ABI call (no GPU needed for the check)."""
    import torch
    s = pflbm.Solver.__new__(pflbm.Solver)
    s.torch, s.device, s._h = torch, torch.device("cuda:0"), None
    for buf in (torch.zeros(16, dtype=torch.uint8), torch.zeros(4, dtype=torch.float32)):
        with pytest.raises(pflbm.PflbmError) as e:
            s.set_state(buf)
        assert e.value.status == -1
