"""Torch-facing binding of libevs (argument marshalling only).

Torch supplies device memory and the current stream; every step of the
computation runs in the library's HIP kernels.
"""

from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import torch

from . import _lib
from ._lib import EvsClip, EvsNet, EvsTnet, check, lib


@dataclass
class Net:
    """EvSNet description: conv3x3 -> BiLIF layers with the given widths."""
    channels: tuple
    theta: float = 0.5
    leak: float = 0.9
    surr_alpha: float = 4.0
    precision: str = "fp32"        # "fp32" | "bf16"
    relaxed: bool = False
    detach_reset: bool = False
    surrogate: str = "sigmoid"      # "sigmoid" or "atan" (the paper's arctangent surrogate)
    # "direct": x is the network input; "rgb_logdiff": x holds T+1 RGB frames
    # and the forward forms the one-channel Eq. (1) input itself
    input: str = "direct"
    lum_scale: float = 255.0
    knee: float = 20.0

    def c(self) -> EvsNet:
        n = EvsNet()
        L = len(self.channels) - 1
        n.n_layers = L
        for i in range(_lib.EVS_MAX_LAYERS + 1):
            n.ch[i] = self.channels[i] if i <= L else 0
        n.theta = self.theta
        n.leak = self.leak
        n.surr_alpha = self.surr_alpha
        n.precision = _lib.EVS_BF16 if self.precision == "bf16" else _lib.EVS_FP32
        n.relaxed = int(self.relaxed)
        n.detach_reset = int(self.detach_reset)
        n.surrogate = {"sigmoid": 0, "atan": 1}[self.surrogate]
        n.input = {"direct": 0, "rgb_logdiff": 1}[self.input]
        n.lum_scale = self.lum_scale
        n.knee = self.knee
        return n

    @property
    def n_layers(self) -> int:
        return len(self.channels) - 1

    @property
    def sum_c(self) -> int:
        return sum(self.channels[1:])


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _clip(x, s_out=None, s_fp32=False, v_state=None, h_trace=None, trace_box=None):
    N, T, _, H, W = x.shape
    c = EvsClip()
    if trace_box is not None:
        for i in range(4):
            c.trace_box[i] = int(trace_box[i])
    c.N, c.T, c.H, c.W = N, T, H, W
    c.x = x.data_ptr()
    c.s_out = s_out.data_ptr() if s_out is not None else None
    c.s_fp32 = int(s_fp32)
    c.v_state = v_state.data_ptr() if v_state is not None else None
    c.h_trace = h_trace.data_ptr() if h_trace is not None else None
    return c


def status_word(device=None) -> torch.Tensor:
    """A zeroed device status word: int32 [EVS_STATUS_WORDS] (NaN count of x,
    NaN count of grad_s, flags, reserved); the library adds to it."""
    return torch.zeros(_lib.EVS_STATUS_WORDS, dtype=torch.int32, device=device or "cuda")


def _check_status(st):
    if st is not None:
        _check_dev(st)
        if st.dtype != torch.int32 or st.numel() < _lib.EVS_STATUS_WORDS:
            raise ValueError("status must be an int32 device tensor of EVS_STATUS_WORDS values")


def _check_dev(*ts):
    for t in ts:
        if t is not None:
            if not t.is_cuda:
                raise ValueError("tensors must live on the GPU")
            if not t.is_contiguous():
                raise ValueError("tensors must be contiguous")


def pack_weights(net: Net, weights, stream=None) -> torch.Tensor:
    L = lib()
    cn = net.c()
    ws = [w.contiguous() for w in weights]
    _check_dev(*ws)
    for w, ci, co in zip(ws, net.channels[:-1], net.channels[1:]):
        if w.dtype != torch.float32 or tuple(w.shape) != (co, ci, 3, 3):
            raise ValueError(f"weight must be float32 [{co},{ci},3,3], got {w.dtype} {tuple(w.shape)}")
    nb = L.evs_packed_weights_bytes(ctypes.byref(cn))
    if nb == ctypes.c_size_t(-1).value:
        check(L.evs_pack_weights(ctypes.byref(cn), None, None, None), "pack_weights")
    packed = torch.empty(nb, dtype=torch.uint8, device=ws[0].device)
    arr = (ctypes.c_void_p * len(ws))(*[w.data_ptr() for w in ws])
    check(L.evs_pack_weights(ctypes.byref(cn), arr, packed.data_ptr(), _stream(stream)), "pack_weights")
    packed._evs_keep = ws       # keep the sources alive until the copy ran
    return packed


def workspace(net: Net, clips, op=_lib.EVS_OP_FORWARD, ckpt_every=0, device=None):
    L = lib()
    cn = net.c()
    arr = (EvsClip * len(clips))(*clips)
    nb = L.evs_workspace_bytes(ctypes.byref(cn), arr, len(clips), ckpt_every, op)
    if nb == ctypes.c_size_t(-1).value:
        raise _lib.EvsError(_lib.EVS_EINVAL, "workspace_bytes")
    if nb == 0:
        return None, 0
    return torch.empty(nb, dtype=torch.uint8, device=device), nb


def forward(net: Net, packed: torch.Tensor, x: torch.Tensor, *, s_fp32: bool = False,
            v_state: torch.Tensor | None = None, trace: bool = False, ckpt_every: int = 0,
            out: torch.Tensor | None = None, stream=None, ws: torch.Tensor | None = None,
            trace_box=None, status: torch.Tensor | None = None):
    """Run the network over x [N,T,Cin,H,W] (float32, on the GPU).

    Returns a dict: "s" [N,T,Cout,H,W] (int8 or float32), "h" (the charged
    potentials of all layers [N,T,sumC,H,W], if trace), "ckpt" (if
    ckpt_every > 0).  v_state [N,sumC,H,W] is read and overwritten in place.
    ``ws`` is an optional preallocated workspace (needed under graph capture,
    where nothing may be allocated).  ``trace_box`` = (y0, x0, h, w) limits
    the trace to that window of the frame.  ``status`` is an optional int32
    device status word (see status_word()).
    """
    if x.dim() == 4:
        x = x.unsqueeze(0)
    _check_dev(x, v_state, packed)
    if x.dtype != torch.float32:
        raise ValueError("x must be float32")
    N, T, C, H, W = x.shape
    if net.input == "rgb_logdiff":
        if C != 3 or T < 2:
            raise ValueError("rgb_logdiff input needs [N, T+1, 3, H, W] frames with T >= 1")
        T -= 1
    elif C != net.channels[0]:
        raise ValueError("x channels do not match the network")
    dev = x.device
    cout = net.channels[-1]
    if out is None:
        out = torch.empty(N, T, cout, H, W, dtype=torch.float32 if s_fp32 else torch.int8, device=dev)
    th, tw = (trace_box[2], trace_box[3]) if trace_box is not None else (H, W)
    h = torch.empty(N, T, net.sum_c, th, tw, dtype=torch.float32, device=dev) if trace else None
    ck = None
    if ckpt_every > 0:
        nseg = (T + ckpt_every - 1) // ckpt_every
        ck = torch.empty(N, nseg, net.sum_c, H, W, dtype=torch.float32, device=dev)
    c = _clip(x, out, s_fp32, v_state, h, trace_box)
    c.T = T
    if ws is None:
        ws, nb = workspace(net, [c], device=dev)
    else:
        nb = ws.numel()
    cn = net.c()
    _check_status(status)
    check(lib().evs_forward(ctypes.byref(cn), packed.data_ptr(), ctypes.byref(c), 1,
                            ck.data_ptr() if ck is not None else None, ckpt_every,
                            ws.data_ptr() if ws is not None else None, nb, _ptr(status), _stream(stream)),
          "forward")
    return {"s": out, "h": h, "ckpt": ck, "_ws": ws}


def forward_batched(net: Net, packed: torch.Tensor, xs, outs, v_states=None, stream=None, ws=None, status=None):
    """One persistent launch over several clips xs[i] [N_i,T_i,Cin,H_i,W_i]."""
    clips = []
    for i, (x, o) in enumerate(zip(xs, outs)):
        v = v_states[i] if v_states is not None else None
        _check_dev(x, o, v)
        clips.append(_clip(x, o, o.dtype == torch.float32, v, None))
    cn = net.c()
    arr = (EvsClip * len(clips))(*clips)
    nb = lib().evs_workspace_bytes(ctypes.byref(cn), arr, len(clips), 0, _lib.EVS_OP_FORWARD)
    if ws is None or ws.numel() < nb:
        ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=xs[0].device)
    _check_status(status)
    check(lib().evs_forward(ctypes.byref(cn), packed.data_ptr(), arr, len(clips), None, 0,
                            ws.data_ptr(), nb, _ptr(status), _stream(stream)), "forward_batched")
    return ws


def tile_count(net: Net) -> int:
    cn = net.c()
    return lib().evs_tile_count(ctypes.byref(cn))


def tile_name(net: Net, tile: int) -> str:
    cn = net.c()
    r = lib().evs_tile_name(ctypes.byref(cn), tile)
    return r.decode() if r else ""


def set_tile(net: Net, tile: int):
    cn = net.c()
    check(lib().evs_set_tile(ctypes.byref(cn), tile), "set_tile")


def autotune(net: Net, H: int, W: int, T: int = 8, stream=None) -> int:
    cn = net.c()
    chosen = ctypes.c_int32(-1)
    check(lib().evs_autotune(ctypes.byref(cn), H, W, T, ctypes.byref(chosen), _stream(stream)), "autotune")
    return chosen.value


def emd_loss(s: torch.Tensor, e: torch.Tensor, lambda_count: float = 0.0, grad: bool = True, stream=None):
    """Bidirectional polarity-split EMD (+ count term); returns (loss, grad_s)."""
    if s.dim() == 4:
        s, e = s.unsqueeze(0), e.unsqueeze(0)
    _check_dev(s, e)
    N, T, C, H, W = s.shape
    loss = torch.empty(1, dtype=torch.float32, device=s.device)
    g = torch.empty_like(s) if grad else None
    c = EvsClip()
    c.N, c.T, c.H, c.W = N, T, H, W
    net = Net((3, C)).c()
    nb = lib().evs_workspace_bytes(ctypes.byref(net), ctypes.byref(c), 1, 0, _lib.EVS_OP_EMD)
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=s.device)
    check(lib().evs_emd_loss(s.data_ptr(), e.data_ptr(), N, T, C, H, W, lambda_count, loss.data_ptr(),
                             g.data_ptr() if g is not None else None, ws.data_ptr(), nb, _stream(stream)),
          "emd_loss")
    return loss, g


def compact_events(s: torch.Tensor, capacity: int | None = None, stream=None, status=None):
    """Dense int8 spikes [T,C,H,W] -> (events uint64 as int64 tensor, count)."""
    _check_dev(s)
    T, C, H, W = s.shape
    if capacity is None:
        capacity = int(s.numel())
    ev = torch.empty(max(capacity, 1), dtype=torch.int64, device=s.device)
    cnt = torch.zeros(1, dtype=torch.int64, device=s.device)
    c = EvsClip()
    c.N, c.T, c.H, c.W = 1, T, H, W
    net = Net((3, C)).c()
    nb = lib().evs_workspace_bytes(ctypes.byref(net), ctypes.byref(c), 1, 0, _lib.EVS_OP_COMPACT)
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=s.device)
    _check_status(status)
    check(lib().evs_compact_events(s.data_ptr(), T, C, H, W, ev.data_ptr(), capacity, cnt.data_ptr(),
                                   ws.data_ptr(), nb, _ptr(status), _stream(stream)), "compact_events")
    return ev, cnt


def logdiff(rgb: torch.Tensor, lum_scale: float = 255.0, knee: float = 20.0, out=None, stream=None):
    """Network input of Eq. (1): RGB frames [N, T+1, 3, H, W] (or [T+1, 3, H, W])
    -> X [N, T, 1, H, W], the temporal difference of the lin-log luminance."""
    _check_dev(rgb)
    if rgb.dim() == 4:
        rgb = rgb.unsqueeze(0)
    N, T1, C, H, W = rgb.shape
    if C != 3 or T1 < 2:
        raise ValueError("logdiff needs [N, T+1, 3, H, W] frames with T >= 1")
    x = out if out is not None else torch.empty(N, T1 - 1, 1, H, W, dtype=torch.float32, device=rgb.device)
    check(lib().evs_logdiff(rgb.data_ptr(), N, T1 - 1, H, W, float(lum_scale), float(knee), x.data_ptr(),
                            _stream(stream)), "logdiff")
    return x


def contrast_events(rgb: torch.Tensor, C: float = 0.2, lum_scale: float = 255.0, knee: float = 20.0, stream=None):
    """Target events of clean frames [N, T, 3, H, W] (or [T, 3, H, W]) -> int8
    [N, T, 2, H, W] ON/OFF counts of an ideal contrast-threshold camera."""
    _check_dev(rgb)
    squeeze = rgb.dim() == 4
    if squeeze:
        rgb = rgb.unsqueeze(0)
    N, T, ch, H, W = rgb.shape
    if ch != 3:
        raise ValueError("contrast_events needs RGB frames")
    e = torch.empty(N, T, 2, H, W, dtype=torch.int8, device=rgb.device)
    check(lib().evs_contrast_events(rgb.data_ptr(), N, T, H, W, float(lum_scale), float(knee), float(C),
                                    e.data_ptr(), _stream(stream)), "contrast_events")
    return e[0] if squeeze else e


@dataclass
class TNet:
    """The paper's temporal EvSNet: kernel-7 Conv1d encoder with 3 residual
    blocks, point-wise projection and one BiLIF unit per pixel."""
    hidden: int = 16
    theta: float = 0.5
    leak: float = 0.9

    def c(self) -> EvsTnet:
        n = EvsTnet()
        n.hidden, n.theta, n.leak = self.hidden, self.theta, self.leak
        return n


def tnet_weight_floats(net: TNet) -> int:
    cn = net.c()
    return int(lib().evs_tnet_weight_floats(ctypes.byref(cn)))


def tnet_forward(net: TNet, weights: torch.Tensor, x: torch.Tensor, debug: bool = False, out=None, stream=None):
    """x [N, T, H, W] (or [N, T, 1, H, W]) float32 -> spikes int8 of the same
    shape; with debug, also [N, T, 7*16 + 2, H, W] float32 activations, u and
    the charged potential (see evs_tnet_forward)."""
    if x.dim() == 5:
        x = x[:, :, 0]
    _check_dev(x, weights)
    if x.dtype != torch.float32 or weights.dtype != torch.float32:
        raise ValueError("x and weights must be float32")
    N, T, H, W = x.shape
    s = out if out is not None else torch.empty(N, T, H, W, dtype=torch.int8, device=x.device)
    d = torch.empty(N, T, 7 * net.hidden + 2, H, W, dtype=torch.float32, device=x.device) if debug else None
    cn = net.c()
    check(lib().evs_tnet_forward(ctypes.byref(cn), weights.data_ptr(), x.data_ptr(), N, T, H, W, s.data_ptr(),
                                 d.data_ptr() if d is not None else None, _stream(stream)), "tnet_forward")
    return s, d


def backward(net: Net, packed, x, ckpt, ckpt_every, grad_s, want_dx=False, want_dv=False, stream=None,
             status=None):
    """BPTT backward; returns (list of dW, dx or None, dv or None)."""
    if x.dim() == 4:
        x = x.unsqueeze(0)
    N, T, C, H, W = x.shape
    dev = x.device
    gws = [torch.empty(co, ci, 3, 3, dtype=torch.float32, device=dev)
           for ci, co in zip(net.channels[:-1], net.channels[1:])]
    dx = torch.empty_like(x) if want_dx else None
    dv = torch.empty(N, net.sum_c, H, W, dtype=torch.float32, device=dev) if want_dv else None
    c = _clip(x)
    cn = net.c()
    nb = lib().evs_workspace_bytes(ctypes.byref(cn), ctypes.byref(c), 1, ckpt_every, _lib.EVS_OP_BACKWARD)
    if nb == ctypes.c_size_t(-1).value:
        raise _lib.EvsError(_lib.EVS_EINVAL, "workspace_bytes(backward)")
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev)
    arr = (ctypes.c_void_p * len(gws))(*[g.data_ptr() for g in gws])
    check(lib().evs_backward(ctypes.byref(cn), packed.data_ptr(), ctypes.byref(c), ckpt.data_ptr(), ckpt_every,
                             grad_s.data_ptr(), arr, dx.data_ptr() if dx is not None else None,
                             dv.data_ptr() if dv is not None else None, ws.data_ptr(), nb, _ptr(status),
                             _stream(stream)),
          "backward")
    return gws, dx, dv


class Graph:
    """A captured sequence of library calls, replayable with one launch.

    Usage::

        g = Graph(stream)            # a non-default torch.cuda.Stream
        with g.capture():
            forward_batched(..., stream=stream)
        g.replay()
    """

    def __init__(self, stream):
        self.stream = stream
        self.exec = None

    def capture(self):
        g = self

        class _Ctx:
            def __enter__(self_inner):
                check(lib().evs_graph_begin(ctypes.c_void_p(g.stream.cuda_stream)), "graph_begin")
                return g

            def __exit__(self_inner, et, ev, tb):
                h = ctypes.c_void_p()
                st = lib().evs_graph_end(ctypes.c_void_p(g.stream.cuda_stream), ctypes.byref(h))
                if et is None:
                    check(st, "graph_end")
                    g.exec = h
                return False

        return _Ctx()

    def replay(self, stream=None):
        s = self.stream if stream is None else stream
        check(lib().evs_graph_launch(self.exec, ctypes.c_void_p(s.cuda_stream)), "graph_launch")

    def __del__(self):
        try:
            if self.exec is not None:
                lib().evs_graph_destroy(self.exec)
        except Exception:
            pass
