"""The C-ABI library loads on the host and exports every entry point that
include/pic.h declares; configuration validation runs without a GPU."""
import ctypes as C
import os
import re

import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared(header="pic.h"):
    txt = open(os.path.join(ROOT, "include", header)).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pic_[a-z_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    from paper_1610_03918_amd import pic
    L = pic.lib()
    names = declared()
    assert len(names) >= 15
    for nm in names:
        assert hasattr(L, nm), nm
    assert set(names) == set(pic.ENTRY_POINTS)
    assert L.pic_version().startswith(b"pic-gfx950")


def test_every_network_symbol_is_exported():
    from paper_1610_03918_amd import unet
    L = unet.lib()
    names = declared("pic_unet.h")
    for nm in names:
        assert hasattr(L, nm), nm
    assert set(names) == set(unet.UNET_ENTRY_POINTS)


def test_network_layer_table_matches_the_oracle():
    """The library's parameter layout (host computation, no GPU) equals the
    oracle network's shapes, in the same order."""
    from oracle import unet as ounet
    from paper_1610_03918_amd import unet
    ys = unet.layers()
    assert [(y["cin"], y["cout"]) for y in ys[:-1]] == ounet.conv_shapes()
    off = 0
    for y in ys[:-1]:
        assert y["w"] == off and y["b"] == off + y["cout"] * 9 * y["cin"]
        off = y["b"] + y["cout"]
    assert ys[-1]["w"] == off and ys[-1]["b"] == off + 16
    assert unet.param_count() == off + 17 == sum(p.size for p in ounet.init_params())
    nb = C.c_size_t(0)
    assert unet.lib().pic_unet_workspace_size(1, 1024, 512, C.byref(nb)) == 0
    assert 2e8 < nb.value < 1.5e9
    assert unet.lib().pic_unet_workspace_size(1, 1020, 512, C.byref(nb)) == -1


def _ws(cfg, cap):
    from paper_1610_03918_amd import pic
    out = C.c_size_t(0)
    st = pic.lib().pic_workspace_size(C.byref(cfg), (C.c_int64 * 2)(*cap), C.byref(out))
    return st, out.value


def test_workspace_size_and_validation():
    from paper_1610_03918_amd.pic import make_config
    w = synth.trench()
    cfg, cc = make_config(w)
    st, n = _ws(cfg, [w.n_particles(0), w.n_particles(1)])
    assert st == 0 and 8e6 < n < 2e8
    bad, cc2 = make_config(w, tile=(12, 16))
    assert _ws(bad, [10, 10])[0] == -1
    wb = synth.bounded_square(n=32)
    wb.edge_cond = (1, 1, 0, 1)              # a bounded edge without a conductor
    cfgb, ccb = make_config(wb)
    assert _ws(cfgb, [10, 10])[0] == -1
    cfgc, ccc = make_config(w, chunk=100)
    assert _ws(cfgc, [10, 10])[0] == -1


def test_recycling_config_validation():
    """Ion recycling needs bulk rows inside the grid that hold no solid cell
    and a non-negative thermal speed; the paper's trench passes."""
    from paper_1610_03918_amd.pic import make_config
    w = synth.paper_trench(15)
    cap = [w.n_particles(0), w.n_particles(1)]
    cfg, cc = make_config(w)
    assert cfg.recycle_rows == 60 and _ws(cfg, cap)[0] == 0
    for rows in (61, w.nx + 1, -1):           # rows into the electrode, past the grid, negative
        bad, cc2 = make_config(w)
        bad.recycle_rows = rows
        assert _ws(bad, cap)[0] == -1, rows
    bad, cc3 = make_config(w)
    bad.recycle_vth = -0.1
    assert _ws(bad, cap)[0] == -1


def test_capacity_beyond_the_fixed_point_charge_bound_is_an_overflow():
    """A capacity above 2^31 - 1 particles per species could exceed the
    int64 node charge (2^32 units per particle): PIC_ERR_OVERFLOW, not a
    generic argument error; 2^31 - 1 itself is accepted."""
    from paper_1610_03918_amd.pic import make_config
    w = synth.trench(nx=64, ny=32, width=4, depth=8, ppc=2)
    cfg, cc = make_config(w)
    assert _ws(cfg, [(1 << 31) - 1, 10])[0] == 0
    assert _ws(cfg, [1 << 31, 10])[0] == -6
    assert _ws(cfg, [10, 1 << 40])[0] == -6
    assert _ws(cfg, [-1, 10])[0] == -1


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors of the C structs have the header's size and field
    offsets (compiled with the host C compiler)."""
    import subprocess
    from paper_1610_03918_amd import pic
    structs = [pic.pic_config, pic.pic_species_buffers, pic.pic_buffers, pic.pic_solve_info, pic.pic_diag,
               pic.pic_hit]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pic.h"', "int main(void) {"]
    want = []
    for st in structs:
        lines.append(f'    printf("%zu\\n", sizeof({st.__name__}));')
        want.append(C.sizeof(st))
        for name, *_ in st._fields_:
            lines.append(f'    printf("%zu\\n", offsetof({st.__name__}, {name}));')
            want.append(getattr(st, name).offset)
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    assert got == want


def test_secondary_emission_configuration_is_validated():
    """Yields outside 0..1, a missing emission speed, a short hit ring or a
    species with a yield that the ring does not log are refused."""
    from paper_1610_03918_amd import pic
    w = synth.trench(nx=48, ny=40, width=6, depth=12, ppc=1, seed=3)
    w.see_yield, w.see_vth = (0.0, 0.5), 0.3
    cfg, cc = pic.make_config(w)
    cap = (C.c_int64 * 2)(1000, 1000)
    nb = C.c_size_t(0)
    assert pic.lib().pic_workspace_size(C.byref(cfg), cap, C.byref(nb)) == 0
    assert cfg.hitlog_capacity >= 65536 and cfg.hitlog_species_mask & 2
    for field, value in (("see_vth", 0.0), ("hitlog_capacity", 1000), ("hitlog_species_mask", 1)):
        bad, _ = pic.make_config(w)
        setattr(bad, field, value)
        assert pic.lib().pic_workspace_size(C.byref(bad), cap, C.byref(nb)) == -1, field
    bad, _ = pic.make_config(w)
    bad.see_yield[1] = 1.5
    assert pic.lib().pic_workspace_size(C.byref(bad), cap, C.byref(nb)) == -1
