"""Host-only checks of the C ABI: the library loads, exports every function
that include/*.h declares, and rejects bad arguments before any launch."""
import ctypes
import glob
import os
import re
import shutil
import subprocess

import pytest

from paper_2204_06633_amd import native

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"\b(lr_[a-z0-9_]+)\s*\(", src):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("lr_orbits_init", "lr_project_links", "lr_tdi_combine"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(native.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings():
    L = native.lib()
    for s in range(6):
        assert L.lr_status_str(s).startswith(b"LR_")
    assert L.lr_abi_version() == native.ABI_VERSION
    hdr = open(os.path.join(ROOT, "include", "lisaresp.h")).read()
    assert "#define LR_ABI_VERSION %d\n" % native.ABI_VERSION in hdr


def _fake_orbits(n=20, dt=1e4, t0=0.0, lmin=8.0, lmax=8.7, rmax=1.6e11):
    o = native.lr_orbits()
    o.t0, o.dt, o.n = t0, dt, n
    o.coef = ctypes.c_void_p(0x1000)          # never dereferenced on the host
    o.L_min, o.L_max, o.R_max = lmin, lmax, rmax
    return o


def test_padding_rules():
    L = native.lib()
    o = _fake_orbits()
    f, b = ctypes.c_int64(), ctypes.c_int64()
    assert L.lr_projection_padding(ctypes.byref(o), 25, 10.0, ctypes.byref(f), ctypes.byref(b)) == 0
    rc = 1.6e11 / 299792458.0
    assert f.value >= (8.7 + rc) / 10.0 + 12 and b.value >= rc / 10.0 + 13
    assert L.lr_tdi_padding(ctypes.byref(o), 25, 2, 10.0, ctypes.byref(f), ctypes.byref(b)) == 0
    assert f.value >= 7 * 8.7 / 10.0 + 12 and b.value >= 13
    assert L.lr_tdi_padding(ctypes.byref(o), 25, 3, 10.0, ctypes.byref(f), ctypes.byref(b)) == 3
    assert L.lr_tdi_padding(ctypes.byref(o), 24, 2, 10.0, ctypes.byref(f), ctypes.byref(b)) == 3


@pytest.mark.parametrize("order,status", [(0, 3), (2, 3), (33, 3)])
def test_bad_order_rejected_before_launch(order, status):
    L = native.lib()
    o = _fake_orbits()
    p = ctypes.c_void_p(0x2000)
    sky = ctypes.c_void_p(0x3000)
    st = L.lr_project_links(ctypes.byref(o), 0.0, 10.0, 1000, p, p, sky, order, 100, 10,
                            ctypes.c_void_p(0x9000000), None)
    assert st == status
    assert L.lr_last_error()


def test_range_and_alias_rejected_before_launch():
    L = native.lib()
    o = _fake_orbits()
    hp, hc = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x200000)
    y = ctypes.c_void_p(0x300000)
    sky = ctypes.c_void_p(0x50000000)
    # stencil would leave h at the front
    assert L.lr_project_links(ctypes.byref(o), 0.0, 10.0, 5000, hp, hc, sky, 25, 3, 10, y,
                              None) == 2
    # output overlapping an input
    assert L.lr_project_links(ctypes.byref(o), 0.0, 10.0, 5000, hp, hc, sky, 25, 200, 10,
                              hp, None) == 1
    # orbit grid does not cover the sample times
    assert L.lr_project_links(ctypes.byref(o), 1e7, 10.0, 5000, hp, hc, sky, 25, 200, 10, y,
                              None) == 2
    # non-finite dt, null sky
    assert L.lr_project_links(ctypes.byref(o), 0.0, float("nan"), 5000, hp, hc, sky, 25,
                              200, 10, y, None) == 1
    assert L.lr_project_links(ctypes.byref(o), 0.0, 10.0, 5000, hp, hc, None, 25, 200, 10, y,
                              None) == 1
    # TDI: unknown channels, generation; too little y before the outputs
    assert L.lr_tdi_combine(ctypes.byref(o), 0.0, 10.0, 500, hp, 2, 25, 7, 100, 10, y, None) == 3
    assert L.lr_tdi_combine(ctypes.byref(o), 0.0, 10.0, 500, hp, 3, 25, 0, 100, 10, y, None) == 3
    assert L.lr_tdi_combine(ctypes.byref(o), 0.0, 10.0, 500, hp, 2, 25, 0, 5, 10, y, None) == 2
    # empty requests are no-ops
    assert L.lr_project_links(ctypes.byref(o), 0.0, 10.0, 5000, hp, hc, sky, 25, 200, 0, y,
                              None) == 0


def test_adjoint_and_likelihood_checks_before_launch():
    L = native.lib()
    o = _fake_orbits()
    a, b, c = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x200000), ctypes.c_void_p(0x300000)
    sky = ctypes.c_void_p(0x50000000)
    # TDI adjoint: too little y before the outputs; bad generation
    assert L.lr_tdi_adjoint(ctypes.byref(o), 0.0, 10.0, 500, 2, 25, 0, 5, 10, a, b, None) == 2
    assert L.lr_tdi_adjoint(ctypes.byref(o), 0.0, 10.0, 500, 5, 25, 0, 100, 10, a, b, None) == 3
    # projection adjoint: sky gradient without h or without workspace
    assert L.lr_project_adjoint(ctypes.byref(o), 0.0, 10.0, 5000, None, None, sky, 25, 200, 10,
                                a, b, c, ctypes.c_void_p(0x70000000), None, 0, None) == 1
    assert L.lr_project_adjoint(ctypes.byref(o), 0.0, 10.0, 5000, a, b, sky, 25, 200, 10,
                                c, ctypes.c_void_p(0x400000), ctypes.c_void_p(0x500000),
                                ctypes.c_void_p(0x70000000), None, 0, None) == 4
    # g_hp aliasing g_hc
    assert L.lr_project_adjoint(ctypes.byref(o), 0.0, 10.0, 5000, None, None, sky, 25, 200, 10,
                                c, a, a, None, None, 0, None) == 1
    assert L.lr_project_adjoint_workspace(1000) >= 2 * 8 * 4
    # likelihood: bad sigma, small workspace
    nb = L.lr_loglike_workspace()
    assert L.lr_loglike(a, b, 10, 0.0, c, None, ctypes.c_void_p(0x600000), nb, None) == 1
    assert L.lr_loglike(a, b, 10, 1.0, c, None, ctypes.c_void_p(0x600000), 8, None) == 4


def test_orbits_init_rejects_bad_input_on_host():
    import numpy as np
    L = native.lib()
    out = native.lr_orbits()
    x = np.zeros((3, 3, 3))
    lt = np.zeros((3, 6))
    dummy = ctypes.c_void_p(0x1000)
    assert L.lr_orbits_init(0.0, 1e4, 3, x.ctypes.data, lt.ctypes.data, dummy, 10 ** 6,
                            ctypes.byref(out), None) == 1
    x = np.zeros((5, 3, 3))
    lt = np.zeros((5, 6))
    assert L.lr_orbits_init(0.0, 1e4, 5, x.ctypes.data, lt.ctypes.data, dummy, 8,
                            ctypes.byref(out), None) == 4
    x[2, 1, 1] = np.nan
    assert L.lr_orbits_init(0.0, 1e4, 5, x.ctypes.data, lt.ctypes.data, dummy, 10 ** 6,
                            ctypes.byref(out), None) == 1


def test_struct_layouts_match_the_header(tmp_path):
    """ctypes mirrors of the header's structs: sizes and field offsets as a C
    compiler lays them out."""
    import subprocess
    structs = {"lr_orbits": native.lr_orbits, "lr_template": native.lr_template,
               "lr_batch": native.lr_batch, "lr_fd_plan": native.lr_fd_plan}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "lisaresp.h"',
             'int main(void) {']
    for name, cls in structs.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (name, name))
        for f in cls._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (name, f[0], name, f[0]))
    lines.append("return 0; }")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    got = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True,
                                                         text=True, check=True).stdout.split("\n")
               if l)
    for name, cls in structs.items():
        assert int(got["%s size" % name]) == ctypes.sizeof(cls), name
        for f in cls._fields_:
            assert int(got["%s %s" % (name, f[0])]) == getattr(cls, f[0]).offset, (name, f[0])


def _batch_templates(rows=3):
    """Three templates (700, 0 and 300 outputs) with 300 h samples of padding
    on each side, laid out one after the other."""
    from paper_2204_06633_amd import inputs
    sp = inputs.make_orbit_samples("keplerian", 1.0e6, 1.0e6 + 1e4)
    tpl, ho, oo = [], 0, 0
    for n in (700, 0, 300):
        tpl.append((ho, n + 600, 300, n, oo))
        ho += n + 600
        oo += rows * n
    arr = (native.lr_template * 3)(*[native.lr_template(*t) for t in tpl])
    return arr, tpl, sp


def test_batch_workspace_and_rejections():
    L = native._batch_lib()
    arr, tpl, sp = _batch_templates()
    o = _fake_orbits(n=sp.n, dt=sp.dt, t0=sp.t0)
    aet = native.CHANNELS["AET"]
    nb = L.lr_batch_workspace(arr, 3, ctypes.byref(o), 10.0, 25, 2, aet, 2, 0, 0, 1)
    assert nb > 0 and nb % 256 == 0
    nb0 = L.lr_batch_workspace(arr, 3, ctypes.byref(o), 10.0, 25, 2, aet, 2, 0, 0, 0)
    assert 0 < nb0 < nb                       # the adjoint adds the link-gradient scratch
    # tile lengths: shorter tiles mean more work items (a larger list)
    n256 = L.lr_batch_workspace(arr, 3, ctypes.byref(o), 10.0, 25, 2, aet, 2, 256, 0, 0)
    n1024 = L.lr_batch_workspace(arr, 3, ctypes.byref(o), 10.0, 25, 2, aet, 2, 1024, 0, 0)
    assert n256 >= nb0 >= n1024 > 0
    # tiles per work item: 1..64, 0 automatic
    for seg in (1, 2, 64):
        assert L.lr_batch_workspace(arr, 3, ctypes.byref(o), 10.0, 25, 2, aet, 2, 0, seg, 0) > 0
    for seg in (-1, 65):
        assert L.lr_batch_workspace(arr, 3, ctypes.byref(o), 10.0, 25, 2, aet, 2, 0, seg, 0) == 0
    # unsupported group size, order, channels, tile; dt too small for a tile
    assert L.lr_batch_workspace(arr, 3, ctypes.byref(o), 10.0, 25, 2, 1, 3, 0, 0, 0) == 0
    assert L.lr_batch_workspace(arr, 3, ctypes.byref(o), 10.0, 24, 2, 1, 2, 0, 0, 0) == 0
    assert L.lr_batch_workspace(arr, 3, ctypes.byref(o), 10.0, 25, 2, 7, 2, 0, 0, 0) == 0
    assert L.lr_batch_workspace(arr, 3, ctypes.byref(o), 10.0, 25, 2, 1, 4, 1024, 0, 0) == 0
    assert L.lr_batch_workspace(arr, 3, ctypes.byref(o), 10.0, 25, 2, 1, 2, 300, 0, 0) == 0
    assert L.lr_batch_workspace(arr, 3, ctypes.byref(o), 0.05, 25, 2, 1, 2, 0, 0, 0) == 0
    assert b"too small" in L.lr_last_error()
    # prepare rejects bad h coverage, overlapping outputs and a short workspace
    # before any device work
    b = native.lr_batch()
    bad = (native.lr_template * 3)(*[native.lr_template(*t) for t in tpl])
    bad[0].n_h = 10
    assert L.lr_batch_prepare(bad, 3, ctypes.byref(o), ctypes.byref(o), 1.0e6, 10.0, 25, 2,
                              1, 2, 0, 0, 0, ctypes.c_void_p(0x1000), 1 << 30, ctypes.byref(b),
                              None) == native.LR_E_RANGE
    bad = (native.lr_template * 3)(*[native.lr_template(*t) for t in tpl])
    bad[2].out_offset = 5
    assert L.lr_batch_prepare(bad, 3, ctypes.byref(o), ctypes.byref(o), 1.0e6, 10.0, 25, 2,
                              1, 2, 0, 0, 0, ctypes.c_void_p(0x1000), 1 << 30, ctypes.byref(b),
                              None) == native.LR_E_ARG
    assert L.lr_batch_prepare(arr, 3, ctypes.byref(o), ctypes.byref(o), 1.0e6, 10.0, 25, 2,
                              1, 2, 0, 0, 0, ctypes.c_void_p(0x1000), 64, ctypes.byref(b),
                              None) == native.LR_E_WORKSPACE


def test_fd_lengths_workspace_and_rejections():
    L = native._fd_lib()
    assert L.lr_fd_length(0) == -1 and L.lr_fd_length(1 + (1 << 24)) == -1
    assert L.lr_fd_length(1) == 4096 and L.lr_fd_length(4096) == 4096
    assert L.lr_fd_length(4097) == 8192 and L.lr_fd_length(3155760) == 1 << 22
    assert L.lr_fd_length(1 << 24) == 1 << 24
    assert L.lr_fd_workspace(3155760, 4, 1) == 0 and L.lr_fd_workspace(100, 3, 0) == 0
    w2, w3 = L.lr_fd_workspace(3155760, 2, 1), L.lr_fd_workspace(3155760, 3, 1)
    N = 1 << 22
    # data spectrum, weights, work and partials: at least 48 + 16 signals bytes per point
    assert w2 >= N * (48 + 16) and w3 >= N * (48 + 32) and w3 > w2
    assert L.lr_fd_workspace(3155760, 3, 4) - w3 >= 3 * 2 * N * 16
    plan = native.lr_fd_plan()
    a, b, c = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x200000), ctypes.c_void_p(0x300000)
    ws = ctypes.c_void_p(0x10000000)
    wsb = L.lr_fd_workspace(5000, 3, 1)
    # bad channel count, dt, stride, null w_t with T, n too large, small workspace
    assert L.lr_fd_prepare(5000, 4, 10.0, a, 5000, b, c, 1, ws, wsb, ctypes.byref(plan), None) == 1
    assert L.lr_fd_prepare(5000, 3, 0.0, a, 5000, b, c, 1, ws, wsb, ctypes.byref(plan), None) == 1
    assert L.lr_fd_prepare(5000, 3, 10.0, a, 4000, b, c, 1, ws, wsb, ctypes.byref(plan), None) == 1
    assert L.lr_fd_prepare(5000, 3, 10.0, a, 5000, b, None, 1, ws, wsb, ctypes.byref(plan),
                           None) == 1
    assert L.lr_fd_prepare((1 << 24) + 1, 3, 10.0, a, 1 << 25, b, c, 1, ws, 1 << 40,
                           ctypes.byref(plan), None) == 3
    assert L.lr_fd_prepare(5000, 3, 10.0, a, 5000, b, c, 1, ws, wsb - 8, ctypes.byref(plan),
                           None) == 4
    # data inside the workspace
    assert L.lr_fd_prepare(5000, 3, 10.0, ctypes.c_void_p(0x10000100), 5000, b, c, 1, ws, wsb,
                           ctypes.byref(plan), None) == 1
    # an unprepared plan is rejected, and so are bad strides and aliasing
    assert L.lr_fd_loglike(ctypes.byref(plan), 1, a, 15000, 5000, b, c, None) == 1
    plan.n, plan.n_fft, plan.log2n, plan.passes, plan.channels = 5000, 8192, 13, 2, 3
    plan.max_batch, plan.ws, plan.ws_bytes = 1, 0x10000000, wsb
    assert L.lr_fd_loglike(ctypes.byref(plan), 1, a, 15000, 4999, b, c, None) == 1
    assert L.lr_fd_loglike(ctypes.byref(plan), 2, a, 14999, 5000, b, c, None) == 1
    assert L.lr_fd_loglike(ctypes.byref(plan), 1, a, 15000, 5000, b, a, None) == 1
    assert L.lr_fd_loglike(ctypes.byref(plan), 1, a, 15000, 5000, None, c, None) == 1
    assert L.lr_fd_loglike(ctypes.byref(plan), 1, a, 15000, 5000, ctypes.c_void_p(0x10000000),
                           c, None) == 1
    assert L.lr_fd_loglike(ctypes.byref(plan), 0, None, 0, 0, None, None, None) == 0


def test_gb_rejections_before_launch():
    L = native._gb_lib()
    p, hp, hc = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x200000), ctypes.c_void_p(0x400000)
    assert L.lr_gb_polarizations(p, 2, 0, 100, 10.0, hp, hc, 99, None) == 1      # stride < n_h
    assert L.lr_gb_polarizations(p, 2, 0, 100, 0.0, hp, hc, 100, None) == 1      # dt
    assert L.lr_gb_polarizations(p, -1, 0, 100, 10.0, hp, hc, 100, None) == 1
    assert L.lr_gb_polarizations(p, 70000, 0, 100, 10.0, hp, hc, 100, None) == 3
    assert L.lr_gb_polarizations(p, 2, 0, 100, 10.0, hp, ctypes.c_void_p(0x200100), 100,
                                 None) == 1                                      # hp / hc overlap
    assert L.lr_gb_polarizations(p, 2, 0, 100, 10.0, None, hc, 100, None) == 1
    assert L.lr_gb_polarizations(p, 0, 0, 100, 10.0, None, None, 100, None) == 0  # nothing to do
    nb = L.lr_gb_adjoint_workspace(2, 3000)
    assert nb >= 2 * 3 * 7 * 8
    w = ctypes.c_void_p(0x800000)
    g = ctypes.c_void_p(0x600000)
    assert L.lr_gb_polarizations_adjoint(p, 2, 0, 3000, 10.0, hp, hc, 3000, g, w, nb - 8,
                                         None) == 4
    assert L.lr_gb_polarizations_adjoint(p, 2, 0, 3000, 10.0, hp, hc, 3000, p, w, nb,
                                         None) == 1                              # g aliases params


# The product defaults of the build-time tuning switches (the values the
# kernel headers define; measured choices, see the headers' comments).
PRODUCT_SWITCHES = {"LR_PROJ_PIPE": 2, "LR_PROJ_MIN_WAVES": 1, "LR_TDI_MIN_WAVES": 4,
                    "LR_FUSED_MIN_WAVES": 2, "LR_FUSED2_MIN_WAVES": 3, "LR_FUSED2W_MIN_WAVES": 2,
                    "LR_TDI_CARRY_MIN_WAVES": 2, "LR_PADJ_CARRY_MIN_WAVES": 2,
                    "LR_TDI_CARRY_KEEP_NU": 1,
                    "LR_TDI_ADJ_FOLD": 1, "LR_PADJ_MIN_WAVES": 1, "LR_SKY_MIN_WAVES": 1,
                    "LR_FD_LS_EXTRA": 1}


def test_product_library_has_the_default_switches():
    """The in-tree library (the one the tests, smoke() and bench.py load
    unless LISARESP_LIB points elsewhere) was built without tuning -D flags:
    a variant build for measurements cannot pass for the product."""
    import os

    from paper_2204_06633_amd import native
    from paper_2204_06633_amd.csrc import build
    assert native.LIB_PATH == build.TARGET or os.environ.get("LISARESP_LIB")
    if os.environ.get("LISARESP_LIB"):
        pytest.skip("LISARESP_LIB selects a variant build")
    assert native.build_config() == PRODUCT_SWITCHES


def test_switch_defaults_in_the_headers():
    """Every switch the library reports is defined once, under #ifndef, in
    a kernel header, with the product value above."""
    import re
    csrc = os.path.join(ROOT, "paper_2204_06633_amd", "csrc")
    found = {}
    for name in os.listdir(csrc):
        if name.endswith((".hpp", ".hip", ".cpp")):
            text = open(os.path.join(csrc, name)).read()
            for m in re.finditer(r"#ifndef (LR_[A-Z0-9_]+)\n#define \1 (\d+)\n#endif", text):
                assert m.group(1) not in found, m.group(1)
                found[m.group(1)] = int(m.group(2))
    assert found == PRODUCT_SWITCHES


def _c_functions(text):
    """(name, body) of every top-level `lr_*` function definition."""
    out = []
    for m in re.finditer(r"\n(?:int|size_t|int64_t|const char\*) (lr_\w+)\([^;{]*\)\s*\{", text):
        depth, i = 1, m.end()
        while depth:
            depth += {"{": 1, "}": -1}.get(text[i], 0)
            i += 1
        out.append((m.group(1), text[m.end():i]))
    return out


def test_every_device_call_opens_a_marker_range():
    """Each C-ABI call that launches kernels or copies opens a roctx range
    named after itself (rocprofv3 --marker-trace), and the library links the
    roctx library."""
    csrc = os.path.join(ROOT, "paper_2204_06633_amd", "csrc")
    device = re.compile(r"\b(run_\w+|launch_\w+|hipMemcpy\w*|hipMemsetAsync|hipLaunchKernelGGL)\(")
    seen = 0
    for f in ("api.cpp", "api_batch.cpp", "api_fd.cpp", "api_gb.cpp", "api_noalloc.hip"):
        for name, body in _c_functions(open(os.path.join(csrc, f)).read()):
            if device.search(body):
                seen += 1
                assert body.lstrip().startswith("LR_CALL_RANGE();"), (f, name)
    assert seen >= 15
    nm = shutil.which("nm")
    if nm:
        syms = subprocess.run([nm, "-D", native.LIB_PATH], capture_output=True, text=True).stdout
        assert "roctxRangePushA" in syms and "roctxRangePop" in syms


def test_segment_rule_in_the_work_list():
    """The plan's segments, seen through the size of the work list: items of
    8 tiles make the list of a long batch ~8 times shorter than items of one;
    the automatic choice takes 8 when the batch keeps >= 2048 items; where
    the TDI halo exceeds what the kernel's rows carry (groups of 4), every
    segment length gives one-tile items."""
    L = native._batch_lib()
    o = _fake_orbits(n=400, dt=1e5)
    aet = native.CHANNELS["AET"]
    n, n_out = 64, 300000                     # 64 templates of 300000 outputs at dt = 10 s
    arr = (native.lr_template * n)(*[native.lr_template(k * (n_out + 4000), n_out + 4000, 2000,
                                                        n_out, 3 * n_out * k) for k in range(n)])

    def ws(group, tile, seg):
        return L.lr_batch_workspace(arr, n, ctypes.byref(o), 10.0, 25, 2, aet, group, tile, seg, 0)

    base = ws(2, 512, 64)                     # a handful of items: everything else
    items = lambda group, tile, seg: ws(group, tile, seg) - base
    i1, i8 = items(2, 512, 1), items(2, 512, 8)
    assert i1 > 6 * i8 > 0
    # automatic: 32 groups x 628 one-tile items = 20096 >= 8 x 2048, so 8
    assert ws(2, 512, 0) == ws(2, 512, 8)
    for seg in (0, 2, 8):
        assert ws(4, 512, seg) == ws(4, 512, 1)
