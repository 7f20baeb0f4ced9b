"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/dn.h, and the host-side validation paths report errors
through dn_last_error()."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dn.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_ ]*?\**\s*\b(dn_[a-z0-9_]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def dn():
    from paper_1811_03882_amd import dn as _dn
    return _dn


def test_every_declared_symbol_is_exported(dn):
    names = declared_functions()
    assert len(names) >= 20, names
    lib = ctypes.CDLL(dn.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # the binding covers the whole ABI
    assert set(names) <= set(dn.SIGNATURES), set(names) - set(dn.SIGNATURES)


def test_channel_pad_and_tiles(dn):
    assert dn.channel_pad(dn.F32, 3) == 4
    assert dn.channel_pad(dn.BF16, 3) == 8
    assert dn.channel_pad(dn.FP8, 125) == 128
    assert dn.channel_pad(7, 3) == -1
    assert dn.tile_count() >= 10
    for t in range(dn.tile_count()):
        bm, bn, wm, wn, mf = dn.tile_info(t)
        assert mf in (16, 32) and bm % (wm * mf) == 0 and bn % (wn * mf) == 0
        assert bm % (16 * wm) == 0 and bn % (16 * wn) == 0
    with pytest.raises(dn.DnError) as e:
        dn.tile_info(dn.tile_count())
    assert e.value.status == dn.DN_EINVAL


def test_conv_sizes_host_arithmetic(dn):
    d = dn.conv_desc(64, 13, 13, 1024, 1024, 3, 1, 1, dtype=dn.BF16, tile=4, splits=1)
    w, v, ws = dn.conv_sizes(d)
    assert w == 1024 * 9 * 1024 * 2 and v == 1024 * 4 and ws == 0
    d = dn.conv_desc(1, 13, 13, 1024, 1024, 3, 1, 1, dtype=dn.F32, tile=0, splits=4)
    assert dn.conv_sizes(d)[2] == 4 * 169 * 1024 * 4
    d = dn.conv_desc(1, 416, 416, 3, 16, 3, 1, 1, dtype=dn.BF16, pool=2, input_nchw=1)
    assert dn.conv_sizes(d) == (16 * 64 * 2, 16 * 4, 0)  # K = 3 filter rows x 16, padded to 64


@pytest.mark.parametrize("kw,status", [
    (dict(pool=2, in_h=13, in_w=13), "DN_EUNSUPPORTED"),      # odd output with fused pool
    (dict(pool=3), "DN_EUNSUPPORTED"),
    (dict(batch=0), "DN_EINVAL"),
    (dict(activation=7), "DN_EINVAL"),
    (dict(dtype=9), "DN_EINVAL"),
    (dict(input_nchw=1, in_c=64), "DN_EUNSUPPORTED"),         # C*k > 16: run does not fit
    (dict(input_nchw=1, in_c=3, ksize=5), "DN_EUNSUPPORTED"), # 5 filter rows > 4
    (dict(input_nchw=1, in_c=5, ksize=3), "DN_EUNSUPPORTED"), # 5 channels pad to 8: 8*3 > 16
    (dict(pool=2, residual=1), "DN_EUNSUPPORTED"),
])
def test_conv_desc_validation(dn, kw, status):
    base = dict(batch=1, in_h=16, in_w=16, in_c=8, cout=8, ksize=3, stride=1, pad=1)
    base.update(kw)
    with pytest.raises(dn.DnError) as e:
        dn.conv_sizes(dn.conv_desc(**base))
    assert e.value.status == getattr(dn, status)
    assert dn.last_error()


def test_net_create_validation_without_gpu(dn):
    import synth
    bad = [synth.conv(16, 3), synth.shortcut(5)]
    with pytest.raises(dn.DnError) as e:
        dn.Net(bad, 3, 32, 32, 1)
    assert e.value.status == dn.DN_EINVAL and "src" in dn.last_error()
    with pytest.raises(dn.DnError) as e:
        dn.Net([synth.conv(16, 3)], 0, 32, 32, 1)
    assert e.value.status == dn.DN_EINVAL
    with pytest.raises(dn.DnError) as e:
        dn.Net([synth.conv(16, 3)], 3, 32, 32, 1, dtype=5)
    assert e.value.status == dn.DN_EINVAL
    with pytest.raises(dn.DnError) as e:
        dn.Net([synth.Layer(9)], 3, 32, 32, 1)
    assert e.value.status == dn.DN_EINVAL


def test_conv_backward_sizes_host_arithmetic(dn):
    # backward-data of a stride-1 3x3 conv 64 -> 128: a forward conv 128 -> 64
    d = dn.conv_desc(2, 20, 18, 64, 128, 3, 1, 1, dtype=dn.BF16)
    w, v, ws = dn.conv_backward_sizes(d)
    assert w == 64 * 9 * 128 * 2 and v == 64 * 4
    # stride 2: the workspace also holds the spread gradient [2][H+2p-k+1][W+2p-k+1][cout_p]
    d = dn.conv_desc(2, 20, 18, 64, 128, 3, 2, 1, dtype=dn.F32)
    w2, v2, ws2 = dn.conv_backward_sizes(d)
    assert w2 == 64 * 9 * 128 * 4 and ws2 >= 2 * 20 * 18 * 128 * 4
    # stem: 3 input channels -> a 3-channel gradient padded to 4 (F32)
    d = dn.conv_desc(1, 416, 416, 3, 16, 3, 1, 1, dtype=dn.F32)
    assert dn.conv_backward_sizes(d)[1] == 4 * 4


@pytest.mark.parametrize("kw,status", [
    (dict(pool=2), "DN_EUNSUPPORTED"),       # fused forms have no backward here
    (dict(residual=1), "DN_EUNSUPPORTED"),
    (dict(input_nchw=1, in_c=3), "DN_EUNSUPPORTED"),
    (dict(dtype=2), "DN_EUNSUPPORTED"),      # FP8
    (dict(pad=3), "DN_EUNSUPPORTED"),        # pad > k - 1
    (dict(cout=0), "DN_EINVAL"),
])
def test_conv_backward_validation(dn, kw, status):
    base = dict(batch=1, in_h=16, in_w=16, in_c=8, cout=8, ksize=3, stride=1, pad=1)
    base.update(kw)
    with pytest.raises(dn.DnError) as e:
        dn.conv_backward_sizes(dn.conv_desc(**base))
    assert e.value.status == getattr(dn, status)
    assert dn.last_error()


def test_backward_op_validation_without_gpu(dn):
    with pytest.raises(dn.DnError) as e:
        dn.leaky_backward(dn.FP8, 16, 1, 1, 0.1, 1)
    assert e.value.status == dn.DN_EUNSUPPORTED
    with pytest.raises(dn.DnError) as e:
        dn.leaky_backward(dn.F32, 6, 1, 1, 0.1, 1)  # not whole 16-byte segments
    assert e.value.status == dn.DN_EINVAL
    with pytest.raises(dn.DnError) as e:
        dn.leaky_backward(dn.F32, 16, 1, 1, 1.5, 1)
    assert e.value.status == dn.DN_EINVAL
    with pytest.raises(dn.DnError) as e:
        dn.maxpool_backward(1, 4, 4, 8, 2, 2, dn.F32, None, 1, 0, 1)
    assert e.value.status == dn.DN_EINVAL
    with pytest.raises(dn.DnError) as e:
        dn.maxpool_backward(1, 4, 4, 8, 2, 0, dn.F32, 1, 1, 0, 1)
    assert e.value.status == dn.DN_EINVAL


def test_backward_net_calls_reject_null_without_gpu(dn):
    assert dn.LIB.dn_input_gradient(None, 0, None, 1, 8, 8, None, None) == dn.DN_EINVAL
    assert dn.LIB.dn_nightmare(None, 0, None, 1, 8, 8, 0.1, 1, None) == dn.DN_EINVAL
    assert dn.LIB.dn_autotune_backward(None, 0, 1, 8, 8, None) == dn.DN_EINVAL
    assert dn.last_error()


def test_leaky_shortcut_rejected(dn):
    import synth
    layers = [synth.conv(16, 3), synth.conv(16, 3), synth.Layer(synth.SHORTCUT, src=0, activation=synth.LEAKY)]
    with pytest.raises(dn.DnError) as e:
        dn.Net(layers, 3, 32, 32, 1)
    assert e.value.status == dn.DN_EUNSUPPORTED


def test_null_safe_destroy(dn):
    dn.LIB.dn_net_destroy(None)
    st = dn.LIB.dn_forward(None, None, 1, 1, 1, None, None)
    assert st == dn.DN_EINVAL


def test_detect_workspace_and_validation(dn):
    assert dn.detect_workspace(2, 5, 20, 13, 13) == ((2 * 20 * 845 * 4 + 255) // 256) * 256 + 2 * 845 * 16
    with pytest.raises(dn.DnError) as e:
        dn.detect_workspace(1, 17, 20, 13, 13)                      # more than 16 anchors
    assert e.value.status == dn.DN_EUNSUPPORTED
    with pytest.raises(dn.DnError) as e:
        dn.detect_workspace(1, 5, 20, 40, 40)                       # 8000 boxes > 4096
    assert e.value.status == dn.DN_EUNSUPPORTED
    with pytest.raises(dn.DnError) as e:
        dn.detect_workspace(0, 5, 20, 13, 13)
    assert e.value.status == dn.DN_EINVAL
    with pytest.raises(dn.DnError) as e:                            # NULL buffers are refused before any launch
        dn.detect(None, 1, 5, 20, 13, 13, [1.0] * 10, 0.2, 0.45, 10, None, 0, None, None, None)
    assert e.value.status == dn.DN_EINVAL


def test_committed_traffic_profile_is_well_formed():
    """The dominant conv's HBM traffic summary (read by bench.py) holds one
    entry per tile config, each above the 63.2 MB the kernel must move."""
    import json
    path = os.path.join(ROOT, "profiles", "conv_dominant_b64_bf16_hbm_traffic.json")
    d = json.load(open(path))
    assert len(d["kernel_source_hash"]) == 16
    entries = d["layer13"]
    assert entries and all(k.startswith("tile") for k in entries)
    for e in entries.values():
        assert e["hbm_bytes_per_launch"] > 63.2e6
        assert abs(e["fetch"]["factor"] - 0.5) < 0.01 and abs(e["write"]["factor"] - 1.0) < 0.01
        assert e["kernel"].startswith("void dnk::conv_igemm_dl<1,")


def test_binding_structs_match_the_header(dn, tmp_path):
    """Every struct the binding passes across the boundary has the header's
    fields, in the header's order, at the header's offsets and size: a C
    program built against include/dn.h prints them (offsetof / sizeof) and
    they are compared with the ctypes mirrors."""
    import subprocess
    pairs = {"dn_layer_desc": dn.LayerDesc, "dn_net_opts": dn.NetOpts, "dn_conv_desc": dn.ConvDesc,
             "dn_pool_desc": dn.PoolDesc, "dn_ga_params": dn.GaParams, "dn_ga_result": dn.GaResult}
    src = open(HEADER).read()
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "dn.h"', "int main(void) {"]
    for cname, cls in pairs.items():
        body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (cname, cname), src, flags=re.S).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        names = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            names += [re.sub(r"[\s*]", "", n).split("[")[0] for n in re.sub(r"^[A-Za-z_ ]+?\s+(?=\**\w+\s*(,|$))", "", decl).split(",")]
        assert [f[0] for f in cls._fields_] == names, (cname, names)
        lines.append('printf("%s .sizeof %%zu\\n", sizeof(%s));' % (cname, cname))
        for n in names:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, n, cname, n))
    lines.append("return 0; }")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line.strip():
            a, b, v = line.split()
            got[(a, b)] = int(v)
    for cname, cls in pairs.items():
        assert got[(cname, ".sizeof")] == ctypes.sizeof(cls), cname
        for n, _ in cls._fields_:
            assert got[(cname, n)] == getattr(cls, n).offset, (cname, n)


def test_halo_kernel_eligibility(dn):
    """Host-side eligibility of the two halo kernels over the GPU tests' shape
    list: every shape either qualifies or is rejected with DN_EUNSUPPORTED
    (never another error); the 9-layer net's c2 / c3 classes qualify for the
    persistent kernel in BF16 and FP8, and its FP32 instances (whose K steps
    exceed the weights it keeps in registers) are rejected."""
    from tests.test_gpu_layers import HALO, HALO_BIG, HALO_TILE, HALO2_TILE
    ok = set()
    for shape in HALO + HALO_BIG:
        b, h, w, cin, cout, k, st, pad, pool, resid = shape
        for dtype in (dn.F32, dn.BF16, dn.FP8):
            for tile in (HALO_TILE, HALO2_TILE):
                d = dn.conv_desc(b, h, w, cin, cout, k, st, pad, 1, 0.1, 2 if pool else 0, resid, dtype,
                                 tile=tile, splits=1)
                try:
                    dn.conv_sizes(d)
                    ok.add((shape, dtype, tile))
                except dn.DnError as e:
                    assert e.status == dn.DN_EUNSUPPORTED, (shape, dtype, tile, e)
    for shape in HALO_BIG:
        for dtype in (dn.BF16, dn.FP8):
            assert (shape, dtype, HALO2_TILE) in ok
        assert (shape, dn.F32, HALO2_TILE) not in ok
    # three 16-channel blocks (48 output channels) run on the earlier halo kernel only
    assert ((1, 17, 19, 16, 48, 3, 2, 1, 0, 0), dn.BF16, HALO_TILE) in ok
    assert ((1, 17, 19, 16, 48, 3, 2, 1, 0, 0), dn.BF16, HALO2_TILE) not in ok
