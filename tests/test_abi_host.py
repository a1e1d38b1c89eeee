"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point that include/evs.h declares, and rejects bad arguments
before enqueuing anything."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "evs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(evs_[a-z0-9_]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def evs():
    import paper_2508_18071_amd as m
    if not os.path.exists(m.LIB_PATH):
        pytest.fail("libevs.so has not been built")
    m.lib()
    return m


def test_header_declares_the_boundary():
    names = _header_functions()
    for required in ("evs_forward", "evs_backward", "evs_emd_loss", "evs_compact_events",
                     "evs_workspace_bytes", "evs_pack_weights", "evs_autotune"):
        assert required in names


def test_library_exports_every_declared_symbol(evs):
    lib = ctypes.CDLL(evs.LIB_PATH)
    for name in _header_functions():
        assert hasattr(lib, name), name
    assert set(_header_functions()) == set(evs.EXPORTED)


def test_status_strings(evs):
    L = evs.lib()
    assert L.evs_status_str(0) == b"ok"
    assert b"invalid" in L.evs_status_str(1)
    assert L.evs_version().startswith(b"evs")


def _net(evs, **kw):
    return evs.Net(**kw).c()


@pytest.mark.parametrize("kw,code", [
    (dict(channels=(3, 16, 16, 2), theta=0.0), 1),
    (dict(channels=(3, 16, 16, 2), leak=1.5), 1),
    (dict(channels=(3,) + (8,) * 8 + (2,)), 1),        # nine layers
    (dict(channels=(3, 16, 33, 16, 2)), 2),             # a hidden layer wider than 32
    (dict(channels=(3, 64, 2)), 2),
    (dict(channels=(3, 16, 3)), 2),
    (dict(channels=(2, 16, 2)), 2),
    (dict(channels=(3, 16, 2), precision="bf16", relaxed=True), 2),
])
def test_forward_rejects_bad_networks_before_launch(evs, kw, code):
    net = _net(evs, **kw)
    c = evs._lib.EvsClip()
    c.N, c.T, c.H, c.W = 1, 4, 8, 8
    c.x = 16  # never dereferenced: validation fails first
    st = evs.lib().evs_forward(ctypes.byref(net), ctypes.c_void_p(16), ctypes.byref(c), 1, None, 0,
                               None, 0, None, None)
    assert st == code
    assert evs.lib().evs_last_error()


def test_forward_rejects_unknown_surrogate(evs):
    net = _net(evs, channels=(3, 16, 2))
    net.surrogate = 2
    c = evs._lib.EvsClip()
    c.N, c.T, c.H, c.W = 1, 4, 8, 8
    c.x = 16
    st = evs.lib().evs_forward(ctypes.byref(net), ctypes.c_void_p(16), ctypes.byref(c), 1, None, 0,
                               None, 0, None, None)
    assert st == 1
    assert b"surrogate" in evs.lib().evs_last_error()


def _header_struct_fields(name):
    import re
    src = open(os.path.join(ROOT, "include", "evs.h")).read()
    body = re.search(r"typedef struct " + name + r" \{(.*?)\} " + name + ";", src, re.S).group(1)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        for part in decl.split(",") if "," in decl and "[" not in decl else [decl]:
            # the declarator's name: the identifier before an optional [size]
            fields.append(re.search(r"(\w+)\s*(?:\[[^\]]*\])?\s*$", part.strip()).group(1))
    return fields


def test_ctypes_structs_mirror_the_header(evs):
    assert _header_struct_fields("evs_net") == [f for f, _ in evs._lib.EvsNet._fields_]
    assert _header_struct_fields("evs_clip") == [f for f, _ in evs._lib.EvsClip._fields_]


def test_forward_rejects_bad_clips_and_workspace(evs):
    L = evs.lib()
    net = _net(evs, channels=(3, 16, 16, 2))
    c = evs._lib.EvsClip()
    c.N, c.T, c.H, c.W = 1, 0, 8, 8
    c.x = 16
    assert L.evs_forward(ctypes.byref(net), ctypes.c_void_p(16), ctypes.byref(c), 1, None, 0, None, 0, None, None) == 1
    c.T = 4
    c.x = None
    assert L.evs_forward(ctypes.byref(net), ctypes.c_void_p(16), ctypes.byref(c), 1, None, 0, None, 0, None, None) == 1
    c.x = 16
    c.v_state = 32           # needs a workspace copy of the initial state
    assert L.evs_forward(ctypes.byref(net), ctypes.c_void_p(16), ctypes.byref(c), 1, None, 0, None, 0, None, None) == 3
    assert L.evs_forward(ctypes.byref(net), None, ctypes.byref(c), 1, None, 0, None, 0, None, None) == 1
    # checkpoints need ckpt_every >= 1
    c.v_state = None
    assert L.evs_forward(ctypes.byref(net), ctypes.c_void_p(16), ctypes.byref(c), 1,
                         ctypes.c_void_p(64), 0, None, 0, None, None) == 1
    c.H = 5000
    assert L.evs_forward(ctypes.byref(net), ctypes.c_void_p(16), ctypes.byref(c), 1, None, 0, None, 0, None, None) == 2


def test_workspace_sizes(evs):
    L = evs.lib()
    net = _net(evs, channels=(3, 16, 16, 2))
    c = evs._lib.EvsClip()
    c.N, c.T, c.H, c.W = 2, 8, 30, 40
    assert L.evs_workspace_bytes(ctypes.byref(net), ctypes.byref(c), 1, 0, 0) == 0
    c.v_state = 16
    assert L.evs_workspace_bytes(ctypes.byref(net), ctypes.byref(c), 1, 0, 0) >= 2 * 34 * 30 * 40 * 4
    assert L.evs_workspace_bytes(ctypes.byref(net), ctypes.byref(c), 1, 0, 99) == ctypes.c_size_t(-1).value


def test_tile_registry(evs):
    for ch, prec in [((3, 16, 16, 2), "fp32"), ((3, 32, 2), "bf16"), ((3, 8, 2), "fp32"), ((1, 1), "fp32")]:
        net = evs.Net(ch, precision=prec)
        n = evs.tile_count(net)
        assert n >= 1
        assert all(evs.tile_name(net, t) for t in range(n))
        with pytest.raises(evs.EvsError):
            evs.set_tile(net, n)


@pytest.mark.parametrize("kw,field,code", [
    (dict(channels=(3, 16, 2), input="rgb_logdiff"), None, 1),            # needs a one-channel net
    (dict(channels=(1, 16, 2), input="rgb_logdiff", precision="bf16"), None, 2),
    (dict(channels=(1, 16, 2), input="rgb_logdiff", knee=0.0), None, 1),
    (dict(channels=(1, 16, 2), input="rgb_logdiff", lum_scale=float("nan")), None, 1),
    (dict(channels=(1, 16, 2)), ("input", 2), 1),
])
def test_forward_rejects_bad_rgb_input(evs, kw, field, code):
    net = _net(evs, **kw)
    if field:
        setattr(net, field[0], field[1])
    c = evs._lib.EvsClip()
    c.N, c.T, c.H, c.W = 1, 4, 8, 8
    c.x = 16
    st = evs.lib().evs_forward(ctypes.byref(net), ctypes.c_void_p(16), ctypes.byref(c), 1, None, 0,
                               None, 0, None, None)
    assert st == code
    assert evs.lib().evs_last_error()


def test_backward_rejects_rgb_input(evs):
    """Training takes the output of evs_logdiff: backward refuses RGB-input nets
    before touching any pointer."""
    net = _net(evs, channels=(1, 16, 2), input="rgb_logdiff")
    c = evs._lib.EvsClip()
    c.N, c.T, c.H, c.W = 1, 4, 8, 8
    c.x = 16
    L = evs.lib()
    assert L.evs_workspace_bytes(ctypes.byref(net), ctypes.byref(c), 1, 2, evs._lib.EVS_OP_BACKWARD) == \
        ctypes.c_size_t(-1).value
    arr = (ctypes.c_void_p * 2)(16, 16)
    st = L.evs_backward(ctypes.byref(net), ctypes.c_void_p(16), ctypes.byref(c), ctypes.c_void_p(16), 2,
                        ctypes.c_void_p(16), arr, None, None, ctypes.c_void_p(16), 1 << 20, None, None)
    assert st == 2
    assert b"evs_logdiff" in L.evs_last_error()


@pytest.mark.parametrize("hidden,theta,leak,N,T,H,W,code", [
    (32, 0.5, 0.9, 1, 4, 4, 4, 2),        # only width 16 is compiled
    (16, 0.0, 0.9, 1, 4, 4, 4, 1),        # theta must be positive
    (16, 0.5, 1.5, 1, 4, 4, 4, 1),        # leak outside [0, 1]
    (16, 0.5, 0.9, 0, 4, 4, 4, 1),        # empty batch
    (16, 0.5, 0.9, 1, 0, 4, 4, 1),        # empty clip
    (16, 0.5, 0.9, 1, 4, 0, 4, 1),
])
def test_tnet_rejects_bad_arguments_before_launch(evs, hidden, theta, leak, N, T, H, W, code):
    """The temporal EvSNet entry point validates its arguments on the host and
    touches no pointer when they are bad (dummy addresses suffice)."""
    net = evs.TNet(hidden=hidden, theta=theta, leak=leak).c()
    st = evs.lib().evs_tnet_forward(ctypes.byref(net), ctypes.c_void_p(16), ctypes.c_void_p(16), N, T, H, W,
                                    ctypes.c_void_p(16), None, None)
    assert st == code
    assert evs.lib().evs_last_error()


def test_tnet_rejects_null_pointers(evs):
    net = evs.TNet().c()
    L = evs.lib()
    assert L.evs_tnet_forward(ctypes.byref(net), None, ctypes.c_void_p(16), 1, 4, 4, 4, ctypes.c_void_p(16),
                              None, None) == 1
    assert L.evs_tnet_forward(ctypes.byref(net), ctypes.c_void_p(16), ctypes.c_void_p(16), 1, 4, 4, 4, None,
                              None, None) == 1
    assert L.evs_tnet_forward(None, ctypes.c_void_p(16), ctypes.c_void_p(16), 1, 4, 4, 4, ctypes.c_void_p(16),
                              None, None) == 1
    assert L.evs_tnet_weight_floats(ctypes.byref(net)) == 16 * 7 + 16 + 6 * (16 * 16 * 7 + 16) + 16 + 1


def test_misaligned_status_word_is_rejected_before_launch(evs):
    """The device status word is optional (NULL records nothing); a pointer
    that cannot hold int32 words is refused on the host."""
    L = evs.lib()
    net = _net(evs, channels=(3, 16, 16, 2))
    c = evs._lib.EvsClip()
    c.N, c.T, c.H, c.W = 1, 4, 8, 8
    c.x = 16
    assert L.evs_forward(ctypes.byref(net), ctypes.c_void_p(16), ctypes.byref(c), 1, None, 0, None, 0,
                         ctypes.c_void_p(18), None) == 1
    assert b"dev_status" in L.evs_last_error()
    arr = (ctypes.c_void_p * 3)(16, 16, 16)
    assert L.evs_backward(ctypes.byref(net), ctypes.c_void_p(16), ctypes.byref(c), ctypes.c_void_p(16), 2,
                          ctypes.c_void_p(16), arr, None, None, ctypes.c_void_p(16), 1 << 30,
                          ctypes.c_void_p(18), None) == 1
    assert L.evs_compact_events(ctypes.c_void_p(16), 4, 2, 8, 8, ctypes.c_void_p(16), 10, ctypes.c_void_p(16),
                                ctypes.c_void_p(16), 1 << 20, ctypes.c_void_p(2), None) == 1


def _gpu_present():
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:
        return False


@pytest.mark.skipif(_gpu_present(), reason="checks the behaviour without a GPU; on a machine with a GPU the call would "
                                           "really run with the placeholder pointers")
def test_no_gpu_reports_hip_error_with_message(evs):
    """Without a GPU, a call with valid arguments gets past validation and
    reports the HIP runtime's failure as EVS_EHIP with a message."""
    L = evs.lib()
    st = L.evs_logdiff(ctypes.c_void_p(256), 1, 2, 4, 4, 255.0, 20.0, ctypes.c_void_p(512), None)
    assert st == 4
    msg = L.evs_last_error()
    assert b"hip" in msg.lower(), msg
    net = _net(evs, channels=(3, 8, 2))
    arr = (ctypes.c_void_p * 2)(256, 512)
    assert L.evs_pack_weights(ctypes.byref(net), arr, ctypes.c_void_p(1024), None) == 4
    assert L.evs_last_error()
