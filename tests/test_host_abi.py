"""CPU-side checks of the library: it loads, exports every symbol the header
declares, the binding's structs and prototypes agree with the header, it rejects
malformed input before touching a device, and its host GF(2) code finds a
correct logical basis."""
import os
import re

import numpy as np
import pytest

from paper_2609_38139_amd import codes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def laim():
    from paper_2609_38139_amd import laim as L
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("liblaim.so is not built: run __graft_entry__.build()")
    L.lib()
    return L


def test_exports_every_declared_symbol(laim):
    hdr = open(os.path.join(ROOT, "include", "laim.h")).read()
    declared = set(re.findall(r"\b(laim_[a-z_0-9]+)\s*\(", hdr))
    assert declared == set(laim.SYMBOLS)
    lib = laim.lib()
    for name in declared:
        assert hasattr(lib, name), name


STRUCTS = {"laim_decode_params": "Params", "laim_resident_cfg": "ResidentCfg",
           "laim_continuous_params": "ContinuousParamsC", "laim_batch_item": "BatchItem",
           "laim_server_event": "ServerEvent", "laim_online_params": "OnlineParamsC"}


def test_binding_structs_match_the_header_layout(tmp_path):
    """Every parameter struct the binding passes by pointer has the size and
    field offsets that a C compiler gives the header's struct."""
    import ctypes as C
    import subprocess
    from paper_2609_38139_amd import laim as L
    hdr = open(os.path.join(ROOT, "include", "laim.h")).read()
    lines = []
    for cname, pyname in STRUCTS.items():
        body = re.search(r"typedef struct \{([^{}]*)\}\s*" + cname + r"\s*;", hdr).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        cfields = re.findall(r"([A-Za-z_][A-Za-z_0-9]*)\s*;", body)
        pyfields = [f[0] for f in getattr(L, pyname)._fields_]
        assert cfields == pyfields, cname
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        lines += [f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));' for f in cfields]
    src = tmp_path / "layout.c"
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"laim.h\"\nint main(void) {\n"
                   + "\n".join(lines) + "\n  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = dict((" ".join(w[:2]), int(w[2])) for w in (ln.split() for ln in out) if w)
    for cname, pyname in STRUCTS.items():
        cls = getattr(L, pyname)
        assert got[f"{cname} size"] == C.sizeof(cls), cname
        for f in cls._fields_:
            assert got[f"{cname} {f[0]}"] == getattr(cls, f[0]).offset, (cname, f[0])


def _c_kind(decl):
    """('ptr', 8) for pointers and the stream handle, else ('int'|'float', size)."""
    decl = decl.strip()
    if "*" in decl or decl.split()[0] == "laim_stream":
        return ("ptr", 8)
    t = " ".join(decl.replace("const ", "").split()[:-1] or decl.split())
    return {"int32_t": ("int", 4), "laim_status": ("int", 4), "int": ("int", 4), "uint64_t": ("int", 8),
            "int64_t": ("int", 8), "size_t": ("int", 8), "double": ("float", 8), "float": ("float", 4),
            "void": None}[t]


def _ctypes_kind(t):
    import ctypes as C
    if t is None:
        return None
    if t in (C.c_void_p, C.c_char_p) or issubclass(t, C._Pointer):
        return ("ptr", 8)
    return ("float" if t in (C.c_float, C.c_double) else "int", C.sizeof(t))


def test_binding_prototypes_match_the_header(laim):
    """Each exported function's argument list and return type, as the
    binding declares them, agree with the header's prototype in count, kind
    (pointer, integer, floating) and width."""
    hdr = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "laim.h")).read(), flags=re.S)
    lib = laim.lib()
    for name in laim.SYMBOLS:
        m = re.search(r"^([A-Za-z_][\w \*]*?)\s*\b" + name + r"\s*\(([^)]*)\)\s*;", hdr, re.M)
        assert m, name
        ret, args = m.group(1), m.group(2).strip()
        cargs = [] if args in ("", "void") else [_c_kind(a) for a in args.split(",")]
        fn = getattr(lib, name)
        assert [_ctypes_kind(t) for t in (fn.argtypes or [])] == cargs, name
        assert _ctypes_kind(fn.restype) == _c_kind(ret + " r"), name


def test_rejects_malformed_csr_without_a_device(laim):
    import ctypes as C
    lib = laim.lib()
    rp = np.array([0, 2, 4], dtype=np.int32)
    bad = np.array([1, 0, 2, 3], dtype=np.int32)  # not ascending
    out = C.c_void_p()
    st = lib.laim_build_tanner(2, 4, rp.ctypes.data_as(C.POINTER(C.c_int32)),
                               bad.ctypes.data_as(C.POINTER(C.c_int32)), 0, None, None, 0, C.byref(out))
    assert st == laim.EINVAL and b"ascending" in lib.laim_last_error()
    col = np.array([0, 1, 2, 7], dtype=np.int32)  # out of range
    st = lib.laim_build_tanner(2, 4, rp.ctypes.data_as(C.POINTER(C.c_int32)),
                               col.ctypes.data_as(C.POINTER(C.c_int32)), 0, None, None, 0, C.byref(out))
    assert st == laim.EINVAL
    # G that does not commute with H
    col = np.array([0, 1, 2, 3], dtype=np.int32)
    grp = np.array([0, 1], dtype=np.int32)
    gcol = np.array([0], dtype=np.int32)
    st = lib.laim_build_tanner(2, 4, rp.ctypes.data_as(C.POINTER(C.c_int32)),
                               col.ctypes.data_as(C.POINTER(C.c_int32)), 1,
                               grp.ctypes.data_as(C.POINTER(C.c_int32)),
                               gcol.ctypes.data_as(C.POINTER(C.c_int32)), 0, C.byref(out))
    assert st == laim.EINVAL and b"commute" in lib.laim_last_error()


def _check_logicals(orc, code, L):
    """L spans ker(G) modulo row(H): right size, commutes with G, and is
    independent modulo row(H) -- checked with the oracle's rank routine."""
    k = code.n - orc.gf2_rank(code.H) - orc.gf2_rank(code.G)
    assert L.shape == (k, code.n)
    if code.G.rows:
        assert not ((code.G.to_dense().astype(np.int64) @ L.T) % 2).any()
    stacked = codes.CSR.from_dense(np.vstack([code.H.to_dense(), L]))
    assert orc.gf2_rank(stacked) == orc.gf2_rank(code.H) + k


@pytest.mark.parametrize("name", ["toric2d:3", "toric2d:6", "bb:6x6", "bb:12x6", "toric3d_point:3",
                                  "toric3d_membrane:3", "rep:7"])
def test_host_logical_basis(laim, orc, name):
    c = codes.by_name(name)
    _check_logicals(orc, c, laim.host_logicals(c))


@pytest.mark.parametrize("name", ["toric2d:5", "toric3d_point:3", "toric3d_point:4",
                                  "toric3d_membrane:3", "toric3d_membrane:4"])
def test_closed_form_logicals(orc, name):
    c = codes.by_name(name)
    _check_logicals(orc, c, c.logicals.to_dense())


def test_homology_test_by_logicals_matches_rank_test(laim, orc):
    """On the L = 3 toric code, 'odd overlap with a logical' decides exactly
    the same shots as the oracle's rank test, over all of ker H plus noise."""
    c = codes.toric_2d(3)
    L = laim.host_logicals(c)
    rng = np.random.default_rng(0)
    r = (rng.random((3000, c.n)) < 0.3).astype(np.uint8)
    s = (r @ c.H.to_dense().T) % 2
    by_logicals = (s.any(1) | ((r @ L.T) % 2).any(1)).astype(np.uint8)
    assert np.array_equal(by_logicals, orc.logical_failure(c, r, np.zeros_like(r)))
