"""The C-ABI library loads and exports every entry point include/ah.h declares
(no GPU needed: nothing is called except ah_status_str / ah_version)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2511_00170_amd", "libah.so")
HDR = os.path.join(ROOT, "include", "ah.h")


def declared():
    txt = open(HDR).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ah_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_path():
    names = declared()
    for n in ["ah_pack", "ah_scan_primers", "ah_pair_amplicons", "ah_tm_nn", "ah_extract", "ah_primers_compile"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libah.so is not built: run python -m paper_2511_00170_amd.build")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    lib.ah_status_str.restype = ctypes.c_char_p
    assert lib.ah_status_str(0) == b"ok"
    assert lib.ah_status_str(2).startswith(b"primer letter")
    assert lib.ah_version() >= 1


def test_binding_names_match_header():
    src = open(os.path.join(ROOT, "paper_2511_00170_amd", "ah.py")).read()
    m = re.search(r"EXPORTED = \[(.*?)\]", src, re.S)
    exported = sorted(re.findall(r'"(ah_[a-z0-9_]+)"', m.group(1)))
    assert exported == declared()


def test_primer_compile_rejects_bad_input_without_gpu():
    """Argument checks happen on the host before any device work."""
    if not os.path.exists(LIB):
        pytest.fail("libah.so is not built")
    lib = ctypes.CDLL(LIB)

    class Spec(ctypes.Structure):
        _fields_ = [("fwd", ctypes.c_char_p), ("rev", ctypes.c_char_p), ("k", ctypes.c_uint32),
                    ("clamp", ctypes.c_uint32), ("min_len", ctypes.c_uint32), ("max_len", ctypes.c_uint32)]

    h = ctypes.c_void_p()
    bad_letter = (Spec * 1)(Spec(b"ACGX", b"ACGT", 1, 1, 10, 100))
    assert lib.ah_primers_compile(bad_letter, 1, ctypes.byref(h)) == 2
    too_long = (Spec * 1)(Spec(b"A" * 33, b"ACGT", 1, 1, 10, 100))
    assert lib.ah_primers_compile(too_long, 1, ctypes.byref(h)) == 3
    clamp = (Spec * 1)(Spec(b"ACGT", b"ACG", 1, 4, 10, 100))
    assert lib.ah_primers_compile(clamp, 1, ctypes.byref(h)) == 3
    window = (Spec * 1)(Spec(b"ACGT", b"ACG", 1, 1, 100, 10))
    assert lib.ah_primers_compile(window, 1, ctypes.byref(h)) == 1


@pytest.mark.parametrize("cfg", [1, 2, 3, 5])
def test_specialised_scan_kernel_compiles_without_gpu(cfg):
    """The hipRTC source generated for a primer set compiles for gfx950 (the
    same headers and options the library uses at run time), in every variant
    the autotuner may pick."""
    if not os.path.exists(LIB):
        pytest.fail("libah.so is not built")
    from paper_2511_00170_amd import ah, synth
    wl = synth.gen_config(cfg, n_seqs=2, len_scale=1e-4)
    variants = ah.JIT_VARIANTS if cfg in (2, 3) else (ah.JIT_DEFAULT_VARIANT,)
    for v in variants:
        assert ah.jit_check(wl.pairs, "gfx950", v) == ah.AH_OK, v
    assert ah.jit_check(wl.pairs, "gfx950", (3, 48)) == ah.AH_E_ARG
    assert ah.jit_check(wl.pairs, "gfx950", (1, 1)) == ah.AH_E_ARG
