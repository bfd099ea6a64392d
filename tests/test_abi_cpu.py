"""The C-ABI library: builds, loads and exports every declared symbol (CPU only)."""
import os
import re
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "epi.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(epi_[a-z_]+)\s*\(", text)))


def test_header_declares_the_abi():
    names = declared()
    for must in ("epi_create", "epi_load_genotypes", "epi_scan", "epi_results", "epi_scan_batch",
                 "epi_server_submit"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2201_02460_amd import epi

    lib = epi.lib()
    out = subprocess.run(["nm", "-D", "--defined-only", epi.LIB_PATH], capture_output=True, text=True, check=True)
    exported = set(re.findall(r" T (epi_\w+)", out.stdout))
    missing = [n for n in declared() if n not in exported]
    assert not missing, f"not exported: {missing}"
    for n in declared():
        assert hasattr(lib, n)
        assert n in epi.SIGNATURES, f"binding lacks {n}"


def test_library_targets_gfx950():
    from paper_2201_02460_amd import epi

    blob = open(epi.LIB_PATH, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in blob


def test_errors_cross_the_abi_as_codes():
    from paper_2201_02460_amd import epi

    # without a usable device the context call fails with a status, not a crash
    rc = epi.lib().epi_create(0, 0, None)
    assert rc == epi.EPI_EINVAL
    assert "null" in epi.epi_last_error()
    assert epi.lib().epi_destroy(None) == epi.EPI_OK


def test_binding_constants_match_the_header():
    """Every #define EPI_* integer the header states has the same value in the binding."""
    from paper_2201_02460_amd import epi

    text = open(HEADER).read()
    defs = dict(re.findall(r"#define\s+(EPI_[A-Z0-9_]+)\s+\(?(-?\d+)\)?", text))
    assert "EPI_MAX_ORDER" in defs and "EPI_BLOCK_SEGMENTED" in defs and "EPI_SERVE_MAX_ORDER" in defs
    for name, value in defs.items():
        assert hasattr(epi, name), f"binding lacks {name}"
        assert getattr(epi, name) == int(value), name
