"""Python binding of the pixel-track library: torch tensors in, torch tensors out.

Each function of this module calls the C entry point of the same name
(`pt_<name>`) with device pointers taken from torch tensors and the current
HIP stream.  PyTorch provides device memory and streams only; all arithmetic
runs in the HIP kernels of libpixeltrack.so.
"""
from __future__ import annotations

import ctypes as ct
from dataclasses import dataclass

import numpy as np
import torch

from . import _abi as A


def _p(t: torch.Tensor | None):
    return ct.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ct.c_void_p(s.cuda_stream)


@dataclass
class Hits:
    """Hit arrays on the device (SoA).  Event e owns [event_offsets[e], event_offsets[e+1])."""
    x: torch.Tensor
    y: torch.Tensor
    z: torch.Tensor
    layer: torch.Tensor           # uint8
    module: torch.Tensor          # int16
    event_offsets: torch.Tensor   # int32 [n_events + 1]

    @property
    def n_hits(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_events(self) -> int:
        return int(self.event_offsets.shape[0] - 1)

    @classmethod
    def from_host(cls, h, device="cuda") -> "Hits":
        """From any object with numpy x, y, z, layer, module, event_offsets."""
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
        return cls(t(h.x), t(h.y), t(h.z), t(h.layer.astype(np.uint8)), t(h.module.astype(np.int16)),
                   t(h.event_offsets.astype(np.int32)))

    def abi(self) -> A.pt_hits:
        h = A.pt_hits()
        h.n_hits = self.n_hits
        h.n_events = self.n_events
        h.event_offsets = self.event_offsets.data_ptr()
        if self.x.dtype == torch.float64:
            h.dtype = A.PT_F64
        elif self.x.dtype == torch.float32:
            h.dtype = A.PT_F32
        else:
            raise TypeError(f"hit coordinates must be float32 or float64, not {self.x.dtype}")
        for a in (self.y, self.z):
            if a.dtype != self.x.dtype or a.shape != self.x.shape:
                raise TypeError("x, y, z must share dtype and shape")
        for name in ("x", "y", "z", "layer", "module", "event_offsets"):
            t = getattr(self, name)
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"hits.{name} must be a contiguous device tensor")
        h.x, h.y, h.z = self.x.data_ptr(), self.y.data_ptr(), self.z.data_ptr()
        h.layer = self.layer.data_ptr()
        h.module = self.module.data_ptr()
        return h


@dataclass
class Cells:
    inner: torch.Tensor
    outer: torch.Tensor
    pair: torch.Tensor
    count: torch.Tensor
    inner_first: torch.Tensor
    inner_count: torch.Tensor

    @property
    def cap(self) -> int:
        return int(self.inner.shape[0])

    @classmethod
    def empty(cls, cap: int, n_hits: int, device="cuda") -> "Cells":
        i32 = dict(dtype=torch.int32, device=device)
        return cls(torch.empty(cap, **i32), torch.empty(cap, **i32), torch.empty(cap, dtype=torch.uint8, device=device),
                   torch.zeros(1, **i32), torch.empty(max(n_hits, 1), **i32), torch.empty(max(n_hits, 1), **i32))

    def abi(self) -> A.pt_cells:
        c = A.pt_cells()
        c.cap = self.cap
        c.inner, c.outer, c.pair = self.inner.data_ptr(), self.outer.data_ptr(), self.pair.data_ptr()
        c.count = self.count.data_ptr()
        c.inner_first, c.inner_count = self.inner_first.data_ptr(), self.inner_count.data_ptr()
        return c

    def valid(self):
        n = min(int(self.count.item()), self.cap)
        return self.inner[:n], self.outer[:n], self.pair[:n]


@dataclass
class Links:
    in_cell: torch.Tensor
    out_cell: torch.Tensor
    count: torch.Tensor
    out_start: torch.Tensor
    out_count: torch.Tensor
    has_inner: torch.Tensor

    @property
    def cap(self) -> int:
        return int(self.in_cell.shape[0])

    @classmethod
    def empty(cls, cap: int, cells_cap: int, device="cuda") -> "Links":
        i32 = dict(dtype=torch.int32, device=device)
        return cls(torch.empty(cap, **i32), torch.empty(cap, **i32), torch.zeros(1, **i32),
                   torch.empty(max(cells_cap, 1), **i32), torch.empty(max(cells_cap, 1), **i32),
                   torch.empty(max(cells_cap, 1), dtype=torch.uint8, device=device))

    def abi(self) -> A.pt_links:
        l = A.pt_links()
        l.cap = self.cap
        l.in_cell, l.out_cell, l.count = self.in_cell.data_ptr(), self.out_cell.data_ptr(), self.count.data_ptr()
        l.out_start, l.out_count = self.out_start.data_ptr(), self.out_count.data_ptr()
        l.has_inner = self.has_inner.data_ptr()
        return l

    def valid(self):
        n = min(int(self.count.item()), self.cap)
        return self.in_cell[:n], self.out_cell[:n]


@dataclass
class Tuplets:
    hits: torch.Tensor        # [cap, 8]
    cells: torch.Tensor       # [cap, 7]
    n: torch.Tensor           # [cap] uint8
    count_raw: torch.Tensor
    kept: torch.Tensor | None
    count: torch.Tensor

    @property
    def cap(self) -> int:
        return int(self.hits.shape[0])

    @classmethod
    def empty(cls, cap: int, device="cuda") -> "Tuplets":
        i32 = dict(dtype=torch.int32, device=device)
        return cls(torch.empty((cap, A.PT_MAX_HITS), **i32), torch.empty((cap, A.PT_MAX_HITS - 1), **i32),
                   torch.empty(cap, dtype=torch.uint8, device=device), torch.zeros(1, **i32),
                   torch.empty(cap, **i32), torch.zeros(1, **i32))

    @classmethod
    def from_rows(cls, hits: torch.Tensor, n: torch.Tensor) -> "Tuplets":
        """Rows given directly (fit without the search): all rows are tracks."""
        dev = hits.device
        cnt = torch.tensor([hits.shape[0]], dtype=torch.int32, device=dev)
        return cls(hits.contiguous(), torch.empty((0, A.PT_MAX_HITS - 1), dtype=torch.int32, device=dev),
                   n.contiguous(), cnt.clone(), None, cnt)

    def abi(self) -> A.pt_ntuplets:
        t = A.pt_ntuplets()
        t.cap = self.cap
        t.hits, t.n = self.hits.data_ptr(), self.n.data_ptr()
        t.cells = self.cells.data_ptr() if self.cells.numel() else None
        t.count_raw, t.count = self.count_raw.data_ptr(), self.count.data_ptr()
        t.kept = self.kept.data_ptr() if self.kept is not None else None
        return t

    def raw(self):
        n = min(int(self.count_raw.item()), self.cap)
        return self.hits[:n], self.n[:n]

    def kept_rows(self):
        n = min(int(self.count.item()), self.cap)
        if self.kept is None:
            return self.hits[:n], self.n[:n]
        rows = self.kept[:n].long()
        return self.hits[rows], self.n[rows]


@dataclass
class Tracks:
    params: torch.Tensor      # [cap, 5]
    chi2: torch.Tensor        # [cap]
    status: torch.Tensor      # [cap] uint8
    cov: torch.Tensor | None = None   # [cap, 15] upper triangles of the parameter covariance

    @classmethod
    def empty(cls, cap: int, precision: int, device="cuda", with_cov: bool = False) -> "Tracks":
        dt = torch.float64 if precision == A.PT_FIT_F64 else torch.float32
        return cls(torch.empty((cap, 5), dtype=dt, device=device), torch.empty(cap, dtype=dt, device=device),
                   torch.empty(cap, dtype=torch.uint8, device=device),
                   torch.empty((cap, 15), dtype=dt, device=device) if with_cov else None)

    def abi(self) -> A.pt_tracks:
        t = A.pt_tracks()
        t.cap = int(self.params.shape[0])
        t.params, t.chi2, t.status = self.params.data_ptr(), self.chi2.data_ptr(), self.status.data_ptr()
        t.cov = self.cov.data_ptr() if self.cov is not None else None
        return t


@dataclass
class Vertices:
    z: torch.Tensor
    var: torch.Tensor
    chi2: torch.Tensor
    ndf: torch.Tensor
    n_tracks: torch.Tensor
    sum_pt2: torch.Tensor
    event_first: torch.Tensor    # [n_events + 1]
    count: torch.Tensor
    track_vertex: torch.Tensor   # [tracks cap]

    @classmethod
    def empty(cls, cap: int, n_events: int, tracks_cap: int, device="cuda") -> "Vertices":
        f64 = dict(dtype=torch.float64, device=device)
        i32 = dict(dtype=torch.int32, device=device)
        return cls(torch.empty(cap, **f64), torch.empty(cap, **f64), torch.empty(cap, **f64), torch.empty(cap, **i32),
                   torch.empty(cap, **i32), torch.empty(cap, **f64), torch.zeros(n_events + 1, **i32),
                   torch.zeros(1, **i32), torch.empty(max(tracks_cap, 1), **i32))

    def abi(self) -> A.pt_vertices:
        v = A.pt_vertices()
        v.cap = int(self.z.shape[0])
        for name in ("z", "var", "chi2", "ndf", "n_tracks", "sum_pt2", "event_first", "count", "track_vertex"):
            setattr(v, name, getattr(self, name).data_ptr())
        return v


def new_status(device="cuda") -> torch.Tensor:
    """A zeroed status block (PT_STATUS_WORDS uint32 words, held as int32)."""
    return torch.zeros(A.PT_STATUS_WORDS, dtype=torch.int32, device=device)


def workspace_size(cfg: A.pt_config, n_hits: int, n_events: int, cells_cap: int, links_cap: int,
                   tuplets_cap: int) -> int:
    n = A.load().pt_workspace_size(ct.byref(cfg), n_hits, n_events, cells_cap, links_cap, tuplets_cap)
    if n == 0:
        raise ValueError("invalid configuration or sizes")
    return int(n)


def new_workspace(nbytes: int, device="cuda") -> torch.Tensor:
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


def _ws(t: torch.Tensor) -> A.pt_workspace:
    w = A.pt_workspace()
    w.ptr = t.data_ptr()
    w.bytes = t.numel()
    return w


# ---------------------------------------------------------------------------
# the five calls

def build_doublets(hits: Hits, cfg: A.pt_config, cells: Cells, status: torch.Tensor, ws: torch.Tensor,
                   stream=None) -> Cells:
    A.check(A.load().pt_build_doublets(ct.byref(hits.abi()), ct.byref(cfg), ct.byref(cells.abi()), _p(status),
                                       _ws(ws), _stream(stream)), "pt_build_doublets")
    return cells


def link_cells(hits: Hits, cfg: A.pt_config, cells: Cells, links: Links, status: torch.Tensor, ws: torch.Tensor,
               stream=None) -> Links:
    A.check(A.load().pt_link_cells(ct.byref(hits.abi()), ct.byref(cfg), ct.byref(cells.abi()),
                                   ct.byref(links.abi()), _p(status), _ws(ws), _stream(stream)), "pt_link_cells")
    return links


def find_ntuplets(hits: Hits, cfg: A.pt_config, cells: Cells, links: Links, tuplets: Tuplets,
                  status: torch.Tensor, ws: torch.Tensor, stream=None) -> Tuplets:
    A.check(A.load().pt_find_ntuplets(ct.byref(hits.abi()), ct.byref(cfg), ct.byref(cells.abi()),
                                      ct.byref(links.abi()), ct.byref(tuplets.abi()), _p(status), _ws(ws),
                                      _stream(stream)), "pt_find_ntuplets")
    return tuplets


def fit_broken_line(hits: Hits, cfg: A.pt_config, tuplets: Tuplets, offsets: torch.Tensor | None, precision: int,
                    tracks: Tracks, status: torch.Tensor, ws: torch.Tensor, stream=None) -> Tracks:
    if offsets is not None and (offsets.dtype != torch.float32 or not offsets.is_contiguous()):
        raise TypeError("module offsets must be a contiguous float32 [n_modules, 3] tensor")
    A.check(A.load().pt_fit_broken_line(ct.byref(hits.abi()), ct.byref(cfg), ct.byref(tuplets.abi()),
                                        _p(offsets), precision, ct.byref(tracks.abi()), _p(status), _ws(ws),
                                        _stream(stream)), "pt_fit_broken_line")
    return tracks


def resolve_ambiguities(hits: Hits, cfg: A.pt_config, cells: Cells, tuplets: Tuplets, precision: int,
                        tracks: Tracks, status: torch.Tensor, ws: torch.Tensor, stream=None):
    """pt_resolve_ambiguities: (selected track indices [cap] int32, count [1])."""
    n = min(tuplets.cap, int(tracks.params.shape[0]))
    sel = torch.empty(max(n, 1), dtype=torch.int32, device=tracks.params.device)
    cnt = torch.zeros(1, dtype=torch.int32, device=tracks.params.device)
    A.check(A.load().pt_resolve_ambiguities(ct.byref(hits.abi()), ct.byref(cfg), ct.byref(cells.abi()),
                                            ct.byref(tuplets.abi()), precision, ct.byref(tracks.abi()), _p(sel),
                                            _p(cnt), _p(status), _ws(ws), _stream(stream)), "pt_resolve_ambiguities")
    return sel, cnt


def find_vertices(hits: Hits, cfg: A.pt_config, tuplets: Tuplets, precision: int, tracks: Tracks,
                  selected: torch.Tensor | None, n_selected: torch.Tensor | None, vertices: Vertices,
                  status: torch.Tensor, ws: torch.Tensor, stream=None) -> Vertices:
    """pt_find_vertices (tracks must carry their covariance)."""
    if tracks.cov is None:
        raise ValueError("pt_find_vertices needs the tracks' covariance (Tracks.empty(..., with_cov=True))")
    A.check(A.load().pt_find_vertices(ct.byref(hits.abi()), ct.byref(cfg), ct.byref(tuplets.abi()), precision,
                                      ct.byref(tracks.abi()), _p(selected), _p(n_selected), ct.byref(vertices.abi()),
                                      _p(status), _ws(ws), _stream(stream)), "pt_find_vertices")
    return vertices


def fit_broken_line_noalloc(hits: Hits, cfg: A.pt_config, tuplets: Tuplets, offsets: torch.Tensor | None,
                            precision: int, tracks: Tracks, status: torch.Tensor, stream=None) -> Tracks:
    """pt_fit_broken_line without a workspace (the library's fixed scratch;
    at most PT_NOALLOC_FIT_MAX_TRACKS tracks; calls on one GPU must not overlap)."""
    if offsets is not None and (offsets.dtype != torch.float32 or not offsets.is_contiguous()):
        raise TypeError("module offsets must be a contiguous float32 [n_modules, 3] tensor")
    A.check(A.load().pt_fit_broken_line_noalloc(ct.byref(hits.abi()), ct.byref(cfg), ct.byref(tuplets.abi()),
                                                _p(offsets), precision, ct.byref(tracks.abi()), _p(status),
                                                _stream(stream)), "pt_fit_broken_line_noalloc")
    return tracks


def fit_broken_line_bwd(hits: Hits, cfg: A.pt_config, tuplets: Tuplets, offsets: torch.Tensor | None,
                        precision: int, g_params: torch.Tensor, g_chi2: torch.Tensor | None,
                        grad_hits: torch.Tensor | None, grad_offsets: torch.Tensor | None, status: torch.Tensor,
                        ws: torch.Tensor, stream=None) -> None:
    want = torch.float64 if precision == A.PT_FIT_F64 else torch.float32
    if g_params.dtype != want or (g_chi2 is not None and g_chi2.dtype != want):
        raise TypeError(f"upstream gradients must be {want} for this precision")
    if grad_hits is not None and grad_hits.dtype != want:
        raise TypeError(f"grad_hits must be {want} [n_hits, 3] for this precision")
    if grad_offsets is not None and grad_offsets.dtype != torch.float64:
        raise TypeError("grad_offsets must be float64 [n_modules, 3]")
    A.check(A.load().pt_fit_broken_line_bwd(ct.byref(hits.abi()), ct.byref(cfg), ct.byref(tuplets.abi()),
                                            _p(offsets), precision, _p(g_params.contiguous()),
                                            _p(g_chi2.contiguous() if g_chi2 is not None else None),
                                            _p(grad_hits), _p(grad_offsets), _p(status), _ws(ws),
                                            _stream(stream)), "pt_fit_broken_line_bwd")


# ---------------------------------------------------------------------------
# convenience: buffers sized once, the whole path in order

class Pipeline:
    """Owns the output buffers, workspace and status block for one workload size."""

    def __init__(self, cfg_dict: dict, *, n_hits: int, n_events: int, cells_cap: int, links_cap: int,
                 tuplets_cap: int, precision: int = A.PT_FIT_F32_F64SOLVE, device="cuda", **perf):
        self.cfg = A.make_config(cfg_dict, **perf)
        self.precision = precision
        self.device = device
        self.cells = Cells.empty(cells_cap, n_hits, device)
        self.links = Links.empty(links_cap, cells_cap, device)
        self.tuplets = Tuplets.empty(tuplets_cap, device)
        self.tracks = Tracks.empty(tuplets_cap, precision, device)
        self.status = new_status(device)
        self.ws = new_workspace(workspace_size(self.cfg, n_hits, n_events, cells_cap, links_cap, tuplets_cap),
                                device)

    def reconstruct(self, hits: Hits, offsets=None, stream=None) -> Tracks:
        build_doublets(hits, self.cfg, self.cells, self.status, self.ws, stream)
        link_cells(hits, self.cfg, self.cells, self.links, self.status, self.ws, stream)
        find_ntuplets(hits, self.cfg, self.cells, self.links, self.tuplets, self.status, self.ws, stream)
        fit_broken_line(hits, self.cfg, self.tuplets, offsets, self.precision, self.tracks, self.status, self.ws,
                        stream)
        return self.tracks

    def backward(self, hits: Hits, g_params, g_chi2, grad_hits, grad_offsets, offsets=None, stream=None) -> None:
        fit_broken_line_bwd(hits, self.cfg, self.tuplets, offsets, self.precision, g_params, g_chi2, grad_hits,
                            grad_offsets, self.status, self.ws, stream)

    def flags(self) -> int:
        return int(self.status[A.PT_ST_FLAGS].item()) & 0xFFFFFFFF


# ---------------------------------------------------------------------------
# batched plans (one hipGraph per step) and kernel timing

class Plan:
    """pt_plan: the whole step captured once into a hipGraph, replayed per call."""

    def __init__(self, cfg: A.pt_config, *, n_hits: int, n_events: int, cells_cap: int, links_cap: int,
                 tuplets_cap: int, precision: int, with_adjoint: bool = False, stages: int = 0):
        """stages: PT_STAGE_* bits; with_adjoint adds PT_STAGE_ADJOINT."""
        self._h = ct.c_void_p()
        stages |= A.PT_STAGE_ADJOINT if with_adjoint else 0
        A.check(A.load().pt_plan_create(ct.byref(cfg), n_hits, n_events, cells_cap, links_cap, tuplets_cap,
                                        precision, stages, ct.byref(self._h)), "pt_plan_create")
        self._keep = None

    def run(self, hits: Hits, cells: Cells, links: Links, tuplets: Tuplets, tracks: Tracks, status: torch.Tensor,
            offsets=None, g_params=None, g_chi2=None, grad_hits=None, grad_offsets=None, selected=None,
            n_selected=None, vertices: "Vertices | None" = None, stream=None) -> None:
        # the structs are rebuilt per call; the plan re-captures only when their contents change
        args = (hits.abi(), cells.abi(), links.abi(), tuplets.abi(), tracks.abi())
        vabi = vertices.abi() if vertices is not None else None
        self._keep = (args, vabi)
        A.check(A.load().pt_plan_run(self._h, *(ct.byref(a) for a in args), _p(offsets), _p(g_params), _p(g_chi2),
                                     _p(grad_hits), _p(grad_offsets), _p(selected), _p(n_selected),
                                     ct.byref(vabi) if vabi is not None else None, _p(status), _stream(stream)),
                "pt_plan_run")

    def __del__(self):
        if getattr(self, "_h", None) and self._h.value:
            A.load().pt_plan_destroy(self._h)
            self._h = ct.c_void_p()


def timing_enable(on: bool = True) -> None:
    A.load().pt_timing_enable(int(on))


def timing_reset() -> None:
    A.load().pt_timing_reset()


def timing_read(kernel: str):
    """(total milliseconds, launches) recorded for a kernel since the last reset."""
    ms = ct.c_double()
    n = ct.c_int64()
    err = A.load().pt_timing_read(kernel.encode(), ct.byref(ms), ct.byref(n))
    if err == A.PT_ERR_ARG:
        return 0.0, 0
    A.check(err, "pt_timing_read")
    return ms.value, n.value
