"""Host-side checks of the C-ABI library: it builds, loads, exports every
symbol include/lt.h declares, and its host-only logic (descriptor validation,
workspace sizing, status strings) behaves; no device call is made."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lt.h")
LIB = os.path.join(ROOT, "paper_2202_02870_amd", "liblt.so")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2202_02870_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lt_[a-z_]+)\s*\(", text)))


def test_header_declares_the_four_operations():
    names = declared_functions()
    for op in ("lt_lproduct", "lt_lsvd", "lt_svt_prox", "lt_complete_pga", "lt_workspace_bytes",
               "lt_create", "lt_destroy"):
        assert op in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_2202_02870_amd import lt
    assert set(declared_functions()) == set(lt.EXPORTED)


def test_status_strings(lib):
    lib.lt_status_string.restype = ctypes.c_char_p
    assert lib.lt_status_string(0) == b"ok"
    assert b"unsupported" in lib.lt_status_string(-3)
    assert b"non-finite" in lib.lt_status_string(-4)


def test_workspace_sizes_host_only():
    from paper_2202_02870_amd import lt
    n_svt = lt.workspace_bytes((144, 176, 3, 50), None, "svt")
    n_pga = lt.workspace_bytes((144, 176, 3, 50), None, "pga")
    nel = 144 * 176 * 150
    assert n_svt >= 2 * nel * 4 and n_pga >= 3 * nel * 4 and n_pga > n_svt
    assert lt.workspace_bytes((144, 176, 3, 50), None, "pga", "bf16x3") > n_pga
    assert lt.workspace_bytes((8, 3, 5), None, "lproduct", shape_b=(3, 7, 5)) > 0
    assert lt.workspace_bytes((16, 12, 4), None, "lsvd") > 0
    # full factors: U 16 x 16, S 16 x 12, V 12 x 12 per slice plus FP64 reflectors
    assert (lt.workspace_bytes((16, 12, 4), None, "lsvd_full") - lt.workspace_bytes((16, 12, 4), None, "lsvd")
            >= 4 * 4 * (16 * 16 + 16 * 12 + 12 * 12) + 4 * 8 * 16 * 12)
    # Fourier modes: SVT and completion (FP32) hold two planes and the real
    # embeddings of one slice per conjugate pair (P = 4: pairs {0}, {1, 3}, {2})
    n_dft = lt.workspace_bytes((8, 8, 4), ("dft",), "svt")
    assert n_dft >= 2 * 8 * 8 * 4 * 4 + 3 * 16 * 16 * 4 * 2
    assert lt.workspace_bytes((8, 8, 4), ("dft",), "pga") > n_dft
    # the economy *_L-SVD: the two planes, the representatives' complex working
    # matrices and columns (P = 4: 3 representatives), factors in two planes
    assert lt.workspace_bytes((8, 6, 4), ("dft",), "lsvd") >= 4 * (2 * 8 * 6 * 4 + 2 * 3 * 2 * 8 * 6
                                                                    + 2 * 4 * (8 * 6 + 6 * 6 + 6 * 6))
    assert lt.workspace_bytes((8, 6, 4), ("dft",), "truncate") > lt.workspace_bytes((8, 6, 4), ("dft",), "lsvd")
    for op, prec in (("svt", "bf16x3"), ("lsvd", "bf16x3"), ("lsvd_full", "f32"), ("truncate", "bf16x3")):
        with pytest.raises(ValueError):      # other operations and BF16 transforms: rejected
            lt.workspace_bytes((8, 8, 4), ("dft",), op, prec)
    # the product under the DFT: real and imaginary planes of A, B and C
    n_lp = lt.workspace_bytes((8, 3, 4), ("dft",), "lproduct", shape_b=(3, 5, 4))
    assert n_lp >= 2 * 4 * 4 * (8 * 3 + 3 * 5 + 8 * 5)
    with pytest.raises(ValueError):
        lt.workspace_bytes((8, 3, 4), ("dft",), "lproduct", "bf16x3", shape_b=(3, 5, 4))
    with pytest.raises(ValueError):          # zero-sized mode
        lt.workspace_bytes((8, 0, 4), None, "svt")


def test_descriptor_layout_matches_c():
    from paper_2202_02870_amd import lt
    assert ctypes.sizeof(lt.Desc) == 4 + 4 * 8 + 4 + 8 * 8 + 8 * 8
    assert ctypes.sizeof(lt.SvdOpts) == 32            # double + 5 int32, padded to 8
    assert ctypes.sizeof(lt.PgaParams) == 4 * 8 + 4 * 4 + 32 + 8   # + start_iter, padded
    assert ctypes.sizeof(lt.PgaReport) == 4 * 4 + 8 + 8 + 8 + 8 + 8
    assert ctypes.sizeof(lt.Profile) == 6 * 8 + 6 * 8 + 8


def test_svt_path_by_shape():
    """The kernel choice is a host decision on the slice shape and options."""
    from paper_2202_02870_amd import lt
    assert lt.svt_path((144, 176, 3, 50)) == "precond"
    assert lt.svt_path((144, 176, 3, 50), precondition=False) == "register"
    assert lt.svt_path((256, 256, 3, 100)) == "register"          # register kernel holds it: no factor
    assert lt.svt_path((600, 256, 2)) == "precond"                  # it does not: 256 x 256 factor
    assert lt.svt_path((256, 256, 3, 100), precondition=False) == "register"
    # beyond the register-resident kernel, the single-problem calls take the
    # wide blocked kernel (LT_WIDE=0: the one-workgroup blocked kernel)
    assert lt.svt_path((512, 512, 3, 64)) == "precond+blocked+wide"
    assert lt.svt_path((512, 512, 3, 64), precondition=False) == "blocked+wide"
    assert lt.svt_path((600, 128, 2)) == "precond"
    assert lt.svt_path((600, 128, 2), precondition=False) == "blocked+wide"
    assert lt.svt_path((128, 600, 2), precondition=False) == "blocked+wide"   # transposed working matrix
    assert lt.svt_path((1024, 64)) == "precond"
    assert lt.svt_path((1024, 64), precondition=False) == "register"
    assert lt.svt_path((2048, 300)) == "precond+blocked+wide"
    assert lt.svt_path((2048, 300), precondition=False) == "blocked+wide"
    os.environ["LT_WIDE"] = "0"
    try:
        assert lt.svt_path((512, 512, 3, 64)) == "precond+blocked"
        assert lt.svt_path((2048, 300), precondition=False) == "blocked"
        assert lt.svt_path((1080, 1920, 3, 2)) == "precond+blocked+wide"   # beyond the one-workgroup kernel
    finally:
        del os.environ["LT_WIDE"]
    assert lt.svt_path((3000, 16)) == "precond"                     # any column length on the factor
    assert lt.svt_path((1, 7)) == "register"                        # n = 1: nothing to factor
    # Fourier modes: the complex Hermitian Jacobi on the complex Cholesky-QR
    # factors (2 min(I1, I2) interleaved real rows) or, unpreconditioned, on the
    # complex slices (2 max(I1, I2) rows) while its register kernel holds them,
    # else the real 2 I1 x 2 I2 embeddings (also with LT_DFT_EMBED=1)
    assert lt.svt_path((100, 80, 4), ("dft",)) == "precond+complex"         # G = 16, 160 -> 16 rows per lane
    assert lt.svt_path((100, 80, 4), ("dft",), precondition=False) == "complex"   # G = 16, 200 -> 16 rows
    assert lt.svt_path((144, 176, 3, 50), ("dft", "dft")) == "precond+complex"    # G = 8, 36 rows per lane
    assert lt.svt_path((144, 176, 3, 50), ("dft", "dft"), precondition=False) == "complex"   # 44 rows
    assert lt.svt_path((190, 192, 2), ("dft",)) == "precond+complex"        # G = 8, 48 rows, one LDS buffer
    assert lt.svt_path((190, 192, 2), ("dft",), precondition=False) == "complex"
    assert lt.svt_path((12, 380, 2), ("dft",), precondition=False) == "complex"   # G = 16, 760 -> 48 rows
    assert lt.svt_path((12, 400, 2), ("dft",)) == "precond+complex"         # the factor: 24 rows
    assert lt.svt_path((12, 400, 2), ("dft",), precondition=False) == "register"  # 800 rows: the 24 x 800 embedding
    assert lt.svt_path((300, 100, 2), ("dft",), precondition=False) == "blocked+wide"   # the 600 x 200 embedding
    assert lt.svt_path((300, 100, 2), ("dft",)) == "precond+complex"
    assert lt.svt_path((192, 192, 2), ("dft",)) == "precond+blocked+wide"   # 96 pairs x 48 rows: beyond the LDS
    assert lt.svt_path((8, 6, 5), ("dft",)) == "precond+complex"
    assert lt.svt_path((8, 1, 5), ("dft",)) == "complex"                    # n = 1: nothing to factor
    os.environ["LT_DFT_EMBED"] = "1"
    try:
        assert lt.svt_path((100, 80, 4), ("dft",)) == "precond"                 # 200 x 160
        assert lt.svt_path((100, 80, 4), ("dft",), precondition=False) == "register"
        assert lt.svt_path((144, 176, 3, 50), ("dft", "dft")) == "precond+blocked+wide"   # 288 x 352
    finally:
        del os.environ["LT_DFT_EMBED"]
    # beyond the one-workgroup blocked kernel: the wide blocked Jacobi (one
    # workgroup per block pair), on the factor up to n = 2304, on the slice up
    # to 2304 rows; the 1080 x 1920 and 2160 x 3840 frames
    assert lt.svt_path((513, 513)) == "precond+blocked+wide"
    assert lt.svt_path((2048, 2048)) == "precond+blocked+wide"
    assert lt.svt_path((1080, 1920, 3, 2)) == "precond+blocked+wide"
    assert lt.svt_path((2160, 3840, 3, 2)) == "precond+blocked+wide"
    assert lt.svt_path((2049, 300), precondition=False) == "blocked+wide"
    assert lt.svt_path((1080, 1920, 3, 2), precondition=False) == "blocked+wide"
    for bad, pc in (((2305, 2305), True), ((3000, 16), False), ((2160, 3840), False), ((4000, 2400), True)):
        with pytest.raises(lt.LtError):
            lt.svt_path(bad, precondition=pc)


def test_pga_warm_by_shape():
    """Completion warm-starts the Jacobi of preconditioned slices of real
    transforms that the register-resident kernel holds with the accumulated
    rotations; the workspace carries those rotations (n x n per slice)."""
    from paper_2202_02870_amd import lt
    assert lt.pga_warm((144, 176, 3, 50))
    assert lt.pga_warm((100, 80, 4))
    assert not lt.pga_warm((144, 176, 3, 50), warm_restart=-1)
    assert not lt.pga_warm((144, 176, 3, 50), precondition=False)
    assert not lt.pga_warm((256, 256, 3, 100))           # no factor: the register kernel takes the slice
    assert not lt.pga_warm((512, 512, 3, 64))            # blocked kernel
    assert not lt.pga_warm((144, 176, 3, 50), ("dft", "dft"))
    assert not lt.pga_warm((1, 7))                       # n = 1: nothing to factor
    shape, n, P = (144, 176, 3, 50), 144, 150
    cold_shape = (256, 256, 3, 100)
    assert (lt.workspace_bytes(shape, None, "pga") - lt.workspace_bytes(shape, None, "svt")
            >= 144 * 176 * P * 4 + P * n * n * 4)
    assert (lt.workspace_bytes(cold_shape, None, "pga") - lt.workspace_bytes(cold_shape, None, "svt")
            < 256 * 256 * 300 * 4 + 300 * 256 * 256 * 4)
