"""CPU checks of the C ABI: the library loads, exports every entry point that
include/lsq.h declares, and rejects bad arguments before touching a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lsq.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lsq_[A-Za-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_1806_02968_amd import lsq
    if not os.path.exists(lsq.LIB_PATH):
        pytest.fail("liblsq.so not built; run __graft_entry__.build()")
    return lsq.lib()


def test_header_declares_the_boundary():
    names = _declared_functions()
    for f in ("lsq_setup", "lsq_solve", "lsq_backward", "lsq_destroy"):
        assert f in names


def test_library_exports_every_declared_symbol(L):
    for name in _declared_functions():
        assert hasattr(L, name), name


def test_binding_list_matches_header():
    from paper_1806_02968_amd import EXPORTS
    assert sorted(EXPORTS) == _declared_functions()


def test_default_options(L):
    from paper_1806_02968_amd import default_options
    o = default_options()
    assert o.mode == 0 and o.tol == 1e-10 and o.fixed_iters == -1 and o.max_replace == 3
    assert o.tie_eps == 2.0 ** -44 and o.max_outer == 30 and o.inner_tol == 1e-5


def test_strerror(L):
    assert L.lsq_strerror(0) == b"ok"
    assert L.lsq_strerror(-2).startswith(b"zero column")
    assert L.lsq_strerror(1) == b"tolerance not reached"
    assert L.lsq_last_error(None) == b""


def test_setup_rejects_bad_arguments_on_the_host(L):
    from paper_1806_02968_amd.lsq import Matrix, LSQ_EINVAL
    ctx = C.c_void_p(0)
    dummy = (C.c_double * 8)()
    addr = C.addressof(dummy)

    def setup(**kw):
        m = Matrix()
        m.format, m.dtype, m.m, m.n, m.ld, m.nnz, m.values = 0, 0, 4, 2, 2, 8, addr
        for k, v in kw.items():
            setattr(m, k, v)
        C_ = kw.pop("C_", 4.0) if "C_" in kw else 4.0
        return L.lsq_setup(C.byref(m), addr, C_, 1, 0, None, None, C.byref(ctx))

    assert setup(m=1, n=2) == LSQ_EINVAL       # m < n
    assert setup(n=0) == LSQ_EINVAL            # n < 1
    assert setup(format=7) == LSQ_EINVAL       # unknown format
    assert setup(dtype=3) == LSQ_EINVAL        # unknown dtype
    assert setup(ld=1) == LSQ_EINVAL           # ld < n
    assert setup(format=1) == LSQ_EINVAL       # CSR without row_ptr/col_idx
    assert setup(values=None) == LSQ_EINVAL    # null values
    m = Matrix()
    m.format, m.dtype, m.m, m.n, m.ld, m.values = 0, 0, 4, 2, 2, addr
    assert L.lsq_setup(C.byref(m), addr, 0.0, 1, 0, None, None, C.byref(ctx)) == LSQ_EINVAL   # C <= 0
    assert L.lsq_setup(C.byref(m), addr, 4.0, -1, 0, None, None, C.byref(ctx)) == LSQ_EINVAL  # sweeps < 0
    assert L.lsq_setup(C.byref(m), None, 4.0, 1, 0, None, None, C.byref(ctx)) == LSQ_EINVAL   # null b
    assert L.lsq_setup(None, addr, 4.0, 1, 0, None, None, C.byref(ctx)) == LSQ_EINVAL         # null A
    assert ctx.value is None


def test_null_context_calls(L):
    assert L.lsq_solve(None, None, None) == -1
    assert L.lsq_solve_many(None, 1, None, 0, None, 0, None) == -1
    assert L.lsq_backward(None, None, None, None, None, None, None) == -1
    assert L.lsq_get_M_nnz(None) == -1
    L.lsq_destroy(None)


def test_oracle_and_library_share_no_source():
    # the oracle is plain C under oracle/, the library HIP under the package
    lib_src = os.path.join(ROOT, "paper_1806_02968_amd", "csrc")
    for f in os.listdir(lib_src):
        text = open(os.path.join(lib_src, f)).read()
        assert "lsq_oracle" not in text and "orc_" not in text
    text = open(os.path.join(ROOT, "oracle", "lsq_oracle.c")).read()
    assert "lsq.h" not in text and "hip" not in text.lower().replace("philox", "")


@pytest.mark.parametrize("struct", ["lsq_options", "lsq_info"])
def test_binding_structs_match_header_layout(struct, tmp_path):
    """The ctypes mirrors of the header's structs have the C compiler's size
    and field offsets (compiled against include/lsq.h with gcc)."""
    import shutil
    import subprocess
    from paper_1806_02968_amd import lsq
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    py = {"lsq_options": lsq.Options, "lsq_info": lsq.Info}[struct]
    names = [f[0] for f in py._fields_]
    src = tmp_path / "layout.c"
    body = "".join('printf("%%s %%zu\\n", "%s", offsetof(%s, %s));' % (f, struct, f) for f in names)
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "lsq.h"\nint main(void){%s'
                   'printf("sizeof %%zu\\n", sizeof(%s));return 0;}\n' % (body, struct))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                       text=True).stdout.splitlines())
    assert int(out["sizeof"]) == C.sizeof(py)
    for f in names:
        assert int(out[f]) == getattr(py, f).offset, f
