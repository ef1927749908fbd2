"""Torch-facing wrappers of the C ABI: device memory and streams come from
torch; every step of the render runs in the HIP library.

Gaussians are passed as a dict of float32 CUDA tensors in the boundary's
structure-of-arrays layout (means [3,N], log_scales [3,N], quats [4,N],
opacity_logits [N], sh [(d+1)^2,3,N]) plus "sh_degree"; cameras as dicts
(w2c 3x4, fx, fy, cx, cy, width, height); options as a dict with the fields
of rgs_options.
"""
from __future__ import annotations

import ctypes as C
from typing import Dict, List, Optional, Sequence

import torch

from . import _lib as L

PARAM_KEYS = ("means", "log_scales", "quats", "opacity_logits", "sh")

DEFAULT_OPTIONS = dict(p_min=1.0 / 255.0, alpha_max=0.99, t_eps=1e-4, near_z=0.2, mip=0, mip_sigma2_px=0.1,
                       background=(0.0, 0.0, 0.0), tile_w=0, tile_h=0,  # 0, 0: tuned shape or 8x16
                       divergence=0)


def _check(lib, ctx, status):
    if status != L.RGS_OK:
        msg = lib.rgs_last_error(ctx)
        raise L.RayGSError(status, msg.decode() if msg else "")


def make_options(opts: Optional[dict] = None) -> L.Options:
    o = dict(DEFAULT_OPTIONS)
    if opts:
        o.update({k: v for k, v in opts.items() if k in DEFAULT_OPTIONS})
    s = L.Options()
    s.p_min, s.alpha_max, s.t_eps, s.near_z = (float(o[k]) for k in ("p_min", "alpha_max", "t_eps", "near_z"))
    s.mip = int(o["mip"])
    s.mip_sigma2_px = float(o["mip_sigma2_px"])
    s.background[:] = [float(v) for v in o["background"]]
    s.tile_w, s.tile_h = int(o["tile_w"]), int(o["tile_h"])
    s.divergence = int(o["divergence"])
    return s


def options_dict(s: L.Options) -> dict:
    return dict(p_min=s.p_min, alpha_max=s.alpha_max, t_eps=s.t_eps, near_z=s.near_z, mip=s.mip,
                mip_sigma2_px=s.mip_sigma2_px, background=tuple(s.background), tile_w=s.tile_w, tile_h=s.tile_h,
                divergence=s.divergence)


def make_cameras(cams: Sequence[dict]):
    arr = (L.Camera * len(cams))()
    for k, c in enumerate(cams):
        w2c = c["w2c"]
        if isinstance(w2c, torch.Tensor):
            w2c = w2c.detach().cpu().double().reshape(-1).tolist()
        else:
            w2c = [float(v) for v in __import__("numpy").asarray(w2c, dtype="float64").reshape(-1)]
        arr[k].world_to_cam[:] = w2c
        arr[k].fx, arr[k].fy, arr[k].cx, arr[k].cy = (float(c[f]) for f in ("fx", "fy", "cx", "cy"))
        arr[k].width, arr[k].height = int(c["width"]), int(c["height"])
    return arr


def _ptr(t: Optional[torch.Tensor]):
    return C.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else C.c_void_p(0)


def make_gaussians(g: Dict[str, torch.Tensor]) -> L.Gaussians:
    n = int(g["opacity_logits"].shape[0])
    deg = int(g["sh_degree"])
    nk = (deg + 1) ** 2
    shapes = dict(means=(3, n), log_scales=(3, n), quats=(4, n), opacity_logits=(n,), sh=(nk, 3, n))
    for k in PARAM_KEYS:
        t = g[k]
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise ValueError(f"{k} must be a contiguous float32 CUDA tensor")
        if tuple(t.shape) != shapes[k]:
            raise ValueError(f"{k} has shape {tuple(t.shape)}, expected {shapes[k]}")
    return L.Gaussians(*(_ptr(g[k]) for k in PARAM_KEYS), n, deg)


def _stream(device) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Renderer:
    """One library context on one GPU; renders batches of views."""

    def __init__(self, device: int = 0, options: Optional[dict] = None, capacity_factor: float = 8.0):
        self.lib = L.load()
        self.device = torch.device("cuda", device)
        h = C.c_void_p()
        st = self.lib.rgs_create(int(device), C.byref(h))
        if st != L.RGS_OK:
            raise L.RayGSError(st, f"rgs_create({device}) failed")
        self.ctx = h
        self.options = dict(DEFAULT_OPTIONS, **(options or {}))
        self.capacity_factor = capacity_factor
        self._capacity: Dict[tuple, int] = {}
        self._ws: Dict[tuple, torch.Tensor] = {}

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.rgs_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- workspace
    def workspace_bytes(self, n, cams, capacity, flags=0, options=None) -> int:
        arr = make_cameras(cams)
        o = make_options(options or self.options)
        out = C.c_size_t()
        _check(self.lib, self.ctx, self.lib.rgs_workspace_size(self.ctx, n, arr, len(cams), C.byref(o), int(capacity),
                                                               int(flags), C.byref(out)))
        return out.value

    def new_workspace(self, n, cams, capacity, flags=0, options=None):
        nbytes = self.workspace_bytes(n, cams, capacity, flags, options)
        buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        ws = L.Workspace(C.c_void_p(buf.data_ptr()), nbytes, int(capacity), int(flags))
        return buf, ws

    def layout(self, n, cams, capacity, flags=0, options=None) -> L.WorkspaceLayout:
        arr = make_cameras(cams)
        o = make_options(options or self.options)
        out = L.WorkspaceLayout()
        _check(self.lib, self.ctx, self.lib.rgs_get_workspace_layout(self.ctx, n, arr, len(cams), C.byref(o),
                                                                     int(capacity), int(flags), C.byref(out)))
        return out

    def default_capacity(self, n, n_views):
        return max(4096, int(self.capacity_factor * max(n, 1) * n_views))

    # ------------------------------------------------------------------ render
    def allocate_outputs(self, cams):
        outs = []
        for c in cams:
            H, W = int(c["height"]), int(c["width"])
            outs.append(dict(rgb=torch.empty((3, H, W), dtype=torch.float32, device=self.device),
                             final_T=torch.empty((H, W), dtype=torch.float32, device=self.device),
                             n_contrib=torch.empty((H, W), dtype=torch.int32, device=self.device)))
        return outs

    @staticmethod
    def _view_outs(outs):
        arr = (L.ViewOut * len(outs))()
        for k, o in enumerate(outs):
            arr[k].rgb, arr[k].final_T, arr[k].n_contrib = _ptr(o["rgb"]), _ptr(o["final_T"]), _ptr(o["n_contrib"])
        return arr

    def render_into(self, g, cams, outs, ws: L.Workspace, options=None):
        """Queue one batched render into caller-provided outputs/workspace."""
        G = make_gaussians(g)
        arr = make_cameras(cams)
        o = make_options(options or self.options)
        _check(self.lib, self.ctx, self.lib.rgs_render(self.ctx, C.byref(G), arr, len(cams), C.byref(o), C.byref(ws),
                                                       self._view_outs(outs), _stream(self.device)))

    def status(self, ws: L.Workspace) -> tuple:
        """(ok, instances needed) after synchronising the current stream."""
        inst = C.c_int64()
        st = self.lib.rgs_render_status(self.ctx, C.byref(ws), _stream(self.device), C.byref(inst))
        if st not in (L.RGS_OK, L.RGS_EOVERFLOW):
            _check(self.lib, self.ctx, st)
        return st == L.RGS_OK, inst.value

    def resolve_options(self, n, cams, options=None) -> dict:
        """Options with tile (0, 0) replaced by the shape the library resolves
        for this configuration now (the context's tuned shape, else 8x16)."""
        o = dict(options or self.options)
        if int(o.get("tile_w", 0)) == 0 and int(o.get("tile_h", 0)) == 0:
            lay = self.layout(n, cams, 1, 0, o)
            o["tile_w"], o["tile_h"] = int(lay.tile_w), int(lay.tile_h)
        return o

    def render(self, g, cams, options=None, flags=0, check=True, keep_workspace=False):
        """Render every camera; returns a list of dicts (rgb [3,H,W], final_T, n_contrib).
        With check=True the instance count is verified (host sync) and the
        workspace grows and the frame is re-rendered on overflow."""
        n = int(g["opacity_logits"].shape[0])
        options = self.resolve_options(n, cams, options)
        key = (n, tuple((int(c["width"]), int(c["height"])) for c in cams), flags,
               tuple(sorted((options or self.options).items())) if isinstance(options or self.options, dict) else None)
        cap = self._capacity.get(key) or self.default_capacity(n, len(cams))
        outs = self.allocate_outputs(cams)
        for _ in range(3):
            if key in self._ws and self._ws[key][1].capacity == cap and not keep_workspace:
                buf, ws = self._ws[key]
            else:
                buf, ws = self.new_workspace(n, cams, cap, flags, options)
                if not keep_workspace:
                    self._ws[key] = (buf, ws)
            self.render_into(g, cams, outs, ws, options)
            if not check:
                break
            ok, need = self.status(ws)
            if ok:
                break
            cap = int(need * 1.25) + 1024
            self._capacity[key] = cap
        self._capacity[key] = cap
        if keep_workspace:
            return outs, (buf, ws)
        return outs

    def backward(self, g, cams, outs, dL_drgb: List[torch.Tensor], ws: L.Workspace, options=None, grads=None):
        """Parameter gradients (dict of tensors shaped like g) for a frame
        rendered into `ws` (which must carry RGS_WS_BACKWARD)."""
        G = make_gaussians(g)
        arr = make_cameras(cams)
        o = make_options(options or self.options)
        if grads is None:
            grads = {k: torch.zeros_like(g[k]) for k in PARAM_KEYS}
        GG = L.GaussianGrads(*(_ptr(grads[k]) for k in PARAM_KEYS))
        dl = [t.contiguous() for t in dL_drgb]
        ptrs = (C.c_void_p * len(dl))(*[t.data_ptr() for t in dl])
        _check(self.lib, self.ctx, self.lib.rgs_render_backward(self.ctx, C.byref(G), arr, len(cams), C.byref(o),
                                                                C.byref(ws), self._view_outs(outs), ptrs, C.byref(GG),
                                                                _stream(self.device)))
        return grads

    def autotune(self, g, cams, ws, outs, reps=5, options=None):
        G = make_gaussians(g)
        arr = make_cameras(cams)
        o = make_options(options or self.options)
        best = L.Options()
        ms = C.c_double()
        _check(self.lib, self.ctx, self.lib.rgs_autotune(self.ctx, C.byref(G), arr, len(cams), C.byref(o),
                                                         C.byref(ws), self._view_outs(outs), int(reps),
                                                         _stream(self.device), C.byref(best), C.byref(ms)))
        return options_dict(best), ms.value

    def autotune_training(self, g, cams, ws, outs, dL_drgb: List[torch.Tensor], reps=3, options=None):
        """Tile shape of the fastest render + backward step (ws must carry
        RGS_WS_BACKWARD); the timed backward passes go into scratch gradients."""
        G = make_gaussians(g)
        arr = make_cameras(cams)
        o = make_options(options or self.options)
        scratch = {k: torch.zeros_like(g[k]) for k in PARAM_KEYS}
        GG = L.GaussianGrads(*(_ptr(scratch[k]) for k in PARAM_KEYS))
        dl = [t.contiguous() for t in dL_drgb]
        ptrs = (C.c_void_p * len(dl))(*[t.data_ptr() for t in dl])
        best = L.Options()
        ms = C.c_double()
        _check(self.lib, self.ctx, self.lib.rgs_autotune_training(
            self.ctx, C.byref(G), arr, len(cams), C.byref(o), C.byref(ws), self._view_outs(outs), ptrs, C.byref(GG),
            int(reps), _stream(self.device), C.byref(best), C.byref(ms)))
        return options_dict(best), ms.value

    # ------------------------------------------------------------------ timing
    def set_stage_timing(self, enable: bool):
        _check(self.lib, self.ctx, self.lib.rgs_set_stage_timing(self.ctx, 1 if enable else 0))

    def stage_times(self):
        names = self.lib.rgs_stage_names().decode().split(";")
        ms = (C.c_double * len(names))()
        frames = C.c_int64()
        self.lib.rgs_stage_times(self.ctx, ms, len(names), C.byref(frames))
        return dict(zip(names, list(ms))), frames.value

    def calibrate(self) -> dict:
        """Measured FP32 FMA TFLOP/s, exp2 Top/s and copy GB/s (rgs_calibrate)."""
        f, e, c = C.c_double(), C.c_double(), C.c_double()
        _check(self.lib, self.ctx, self.lib.rgs_calibrate(self.ctx, _stream(self.device), C.byref(f), C.byref(e),
                                                          C.byref(c)))
        return {"fma_tflops": f.value, "exp2_tops": e.value, "copy_gbs": c.value}

    def downsample(self, img: torch.Tensor, factor: int) -> torch.Tensor:
        """Box average of factor x factor blocks of a [P][H f][W f] float32
        device image (rgs_downsample_box): [P][H][W]."""
        assert img.dtype == torch.float32 and img.is_cuda and img.dim() == 3
        img = img.contiguous()
        p, hs, ws = img.shape
        assert hs % factor == 0 and ws % factor == 0
        out = torch.empty((p, hs // factor, ws // factor), dtype=torch.float32, device=img.device)
        _check(self.lib, self.ctx, self.lib.rgs_downsample_box(self.ctx, C.c_void_p(img.data_ptr()), ws // factor,
                                                               hs // factor, int(factor), p,
                                                               C.c_void_p(out.data_ptr()), _stream(self.device)))
        return out

    def set_view_clocks(self, stamps: Optional[torch.Tensor]):
        """Per-view completion clocks of later render_into calls: `stamps` is
        an int64 device tensor of max_views + 1 entries (None turns them off);
        see view_latencies_ms."""
        if stamps is None:
            _check(self.lib, self.ctx, self.lib.rgs_set_view_clocks(self.ctx, None, 0))
            return
        assert stamps.dtype == torch.int64 and stamps.is_cuda and stamps.is_contiguous()
        _check(self.lib, self.ctx, self.lib.rgs_set_view_clocks(self.ctx, C.c_void_p(stamps.data_ptr()),
                                                                stamps.numel() - 1))

    def view_latencies_ms(self, stamps: torch.Tensor, n_views: int):
        """Milliseconds from the frame start to each view's last finished
        compositing work item, from a stamps tensor written by a render."""
        hz = self.lib.rgs_wall_clock_hz(self.ctx)
        s = stamps[: n_views + 1].cpu().numpy().astype("float64")
        return list((s[1:] - s[0]) * 1e3 / hz)


class BatchRenderer:
    """A fixed batch of views rendered by one HIP-graph replay per frame."""

    def __init__(self, renderer: Renderer, n: int, sh_degree: int, cams, capacity: int, options=None, flags=0):
        self.r = renderer
        self.lib = renderer.lib
        self.options = dict(renderer.options, **(options or {}))
        arr = make_cameras(cams)
        o = make_options(self.options)
        nbytes = C.c_size_t()
        plan = C.c_void_p()
        _check(self.lib, renderer.ctx, self.lib.rgs_batch_plan(renderer.ctx, int(n), int(sh_degree), arr, len(cams),
                                                               C.byref(o), int(capacity), int(flags), C.byref(nbytes),
                                                               C.byref(plan)))
        self.plan = plan
        self.buf = torch.empty(nbytes.value, dtype=torch.uint8, device=renderer.device)
        self.ws = L.Workspace(C.c_void_p(self.buf.data_ptr()), nbytes.value, int(capacity), int(flags))
        self.outs = renderer.allocate_outputs(cams)
        self._outs_arr = Renderer._view_outs(self.outs)

    def launch(self, g, cams):
        G = make_gaussians(g)
        arr = make_cameras(cams)
        _check(self.lib, self.r.ctx, self.lib.rgs_batch_launch(self.plan, C.byref(G), arr, C.byref(self.ws),
                                                               self._outs_arr, _stream(self.r.device)))
        return self.outs

    def status(self) -> tuple:
        """(fits, instances needed) of the last launch (rgs_batch_status)."""
        inst = C.c_int64()
        st = self.lib.rgs_batch_status(self.plan, C.byref(inst))
        if st not in (L.RGS_OK, L.RGS_EOVERFLOW):
            _check(self.lib, self.r.ctx, st)
        return st == L.RGS_OK, inst.value

    def close(self):
        if getattr(self, "plan", None):
            self.lib.rgs_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class RenderFunction(torch.autograd.Function):
    """Differentiable batched render: returns one rgb tensor per camera."""

    @staticmethod
    def forward(ctx, renderer: Renderer, cams, options, sh_degree, means, log_scales, quats, opacity_logits, sh):
        g = dict(means=means.contiguous(), log_scales=log_scales.contiguous(), quats=quats.contiguous(),
                 opacity_logits=opacity_logits.contiguous(), sh=sh.contiguous(), sh_degree=sh_degree)
        # the backward must see the forward's tile shape
        options = renderer.resolve_options(int(means.shape[1]), cams, options)
        outs, (buf, ws) = renderer.render(g, cams, options, flags=L.RGS_WS_BACKWARD, check=True, keep_workspace=True)
        ctx.renderer, ctx.cams, ctx.options, ctx.g, ctx.outs, ctx.ws_buf, ctx.ws = renderer, cams, options, g, outs, buf, ws
        return tuple(o["rgb"] for o in outs)

    @staticmethod
    def backward(ctx, *grad_rgb):
        dl = [(gr if gr is not None else torch.zeros_like(o["rgb"])).contiguous() for gr, o in zip(grad_rgb, ctx.outs)]
        grads = ctx.renderer.backward(ctx.g, ctx.cams, ctx.outs, dl, ctx.ws, ctx.options)
        return (None, None, None, None, grads["means"], grads["log_scales"], grads["quats"], grads["opacity_logits"],
                grads["sh"])


def render(renderer: Renderer, g: Dict[str, torch.Tensor], cams, options=None):
    """Differentiable render of all cameras; returns a list of [3,H,W] tensors."""
    return list(RenderFunction.apply(renderer, cams, options, int(g["sh_degree"]), g["means"], g["log_scales"],
                                     g["quats"], g["opacity_logits"], g["sh"]))
