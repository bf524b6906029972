"""The C-ABI library loads and exports every entry point include/dme.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dme.h")
LIB = os.path.join(ROOT, "paper_1805_08990_amd", "libdme.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:int|void|const char\s*\*)\s*\**\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def ensure_built():
    if not os.path.exists(LIB):
        from paper_1805_08990_amd.build import build
        build()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("dme_create", "dle_solve", "dre_solve", "dme_expm", "dme_compress",
                     "dme_riccati", "dme_syev", "dme_gemm_f64", "dme_solver_step"):
        assert required in names


def test_library_exports_every_declared_symbol():
    ensure_built()
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_strerror_without_gpu():
    ensure_built()
    lib = ctypes.CDLL(LIB)
    lib.dme_strerror.restype = ctypes.c_char_p
    assert lib.dme_strerror(0) == b"ok"
    assert lib.dme_strerror(-3) == b"rank exceeds max_rank"


def test_binding_imports_and_marshals_options():
    ensure_built()
    from paper_1805_08990_amd import _binding as b
    o = b.SolveOptions(T=0.1, h=1e-3, tol=1e-10, scheme="lie", split="F1F2", precision="mixed",
                       quad_nodes=5, max_rank=64).to_c()
    assert (o.scheme, o.split, o.precision, o.quad_nodes, o.max_rank) == (0, 1, 1, 5, 64)
    assert ctypes.sizeof(b.Opts) == 3 * 8 + 4 * 4 + 8 + 8  # action + padding
    assert ctypes.sizeof(b.Problem) == 4 * 8 + 11 * 8
