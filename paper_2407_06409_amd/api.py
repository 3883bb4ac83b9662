"""Python face of the lMBD library: marshals arguments to the C ABI.

Every step of the method runs in the HIP kernels of ``liblmbd.so``; torch is
used only for device memory and the current stream.
"""
import ctypes
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as C


@dataclass
class MethodParams:
    """Parameters shared by every structure of a call (lengths in Angstrom, Ha)."""
    omega: Sequence[float]
    weight: Sequence[float]
    beta: float = 0.83
    damp_d: float = 6.0
    r_buf: float = 0.5
    r_inner: float = 2.0
    n_max: int = 6
    c_n: Optional[Sequence[float]] = None
    precision: str = "fp64"
    scs_freq: str = "exact"      # "exact" or "lorentz" (two-point model, Sec. III.C)
    omega_ref: float = 0.0       # reference frequency of the two-point model, Ha
    force_model: str = "exact"   # "exact" (gradient of sum_k w_k E_k) or "paper" (Sec. III.D approximation)
    cn_mode: str = "series"      # "series" (c_n above) or "fit" (per atom and node, Sec. III.A)
    lanczos_steps: int = 20      # Lanczos steps of the fit and of the spectrum output

    def to_c(self):
        om = np.ascontiguousarray(self.omega, dtype=np.float64)
        wt = np.ascontiguousarray(self.weight, dtype=np.float64)
        keep = [om, wt]
        cn = None
        if self.c_n is not None:
            cn = np.ascontiguousarray(self.c_n, dtype=np.float64)
            keep.append(cn)
        p = C.Params(self.beta, self.damp_d, self.r_buf, self.r_inner, int(self.n_max),
                     cn.ctypes.data_as(C._dp) if cn is not None else None, int(om.shape[0]),
                     om.ctypes.data_as(C._dp), wt.ctypes.data_as(C._dp),
                     C.LMBD_MIXED if self.precision == "mixed" else C.LMBD_FP64,
                     {"exact": C.LMBD_SCS_EXACT, "lorentz": C.LMBD_SCS_LORENTZ}[self.scs_freq],
                     float(self.omega_ref),
                     {"exact": C.LMBD_FORCES_EXACT, "paper": C.LMBD_FORCES_PAPER}[self.force_model],
                     {"series": C.LMBD_CN_SERIES, "fit": C.LMBD_CN_FIT}[self.cn_mode], int(self.lanczos_steps))
        return p, keep


def species_array(table):
    t = np.asarray(table, dtype=np.float64).reshape(-1, 3)
    arr = (C.Species * t.shape[0])()
    for i, (a, c6, r0) in enumerate(t):
        arr[i] = C.Species(a, c6, r0)
    return arr, t.shape[0]


class Context:
    """Owns one library context (device workspaces) on one GPU."""

    def __init__(self, device: int = 0, memory_budget: int = 0):
        self.lib = C.lib()
        h = ctypes.c_void_p()
        st = self.lib.lmbd_create(int(device), ctypes.byref(h))
        if st != 0:
            raise C.LmbdError(st, f"lmbd_create(device={device})")
        self.handle = h
        self.device = device
        if memory_budget:
            self.set_memory_budget(memory_budget)

    def set_memory_budget(self, nbytes: int):
        st = self.lib.lmbd_set_memory_budget(self.handle, ctypes.c_size_t(int(nbytes)))
        if st != 0:
            raise C.LmbdError(st)

    def set_mbd_product(self, mode: str = "auto"):
        """'auto', 'dense' (T_LR stored, matrix-core products) or 'sparse' (coupled pairs only)."""
        code = {"auto": C.LMBD_MBD_AUTO, "dense": C.LMBD_MBD_DENSE, "sparse": C.LMBD_MBD_SPARSE}[mode]
        st = self.lib.lmbd_set_mbd_product(self.handle, code)
        if st != 0:
            raise C.LmbdError(st, self.last_error())

    def set_profiling(self, on: bool = True):
        st = self.lib.lmbd_set_profiling(self.handle, 1 if on else 0)
        if st != 0:
            raise C.LmbdError(st, self.last_error())

    def stage_times(self) -> dict:
        """Milliseconds per stage of the last call (HIP events on the call's stream)."""
        arr = (ctypes.c_double * C.N_STAGES)()
        st = self.lib.lmbd_stage_times(self.handle, arr)
        if st != 0:
            raise C.LmbdError(st)
        return {self.lib.lmbd_stage_name(i).decode(): arr[i] for i in range(C.N_STAGES)}

    def last_error(self) -> str:
        return (self.lib.lmbd_last_error(self.handle) or b"").decode()

    def close(self):
        if getattr(self, "handle", None):
            self.lib.lmbd_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_ctx = {}


def default_context(device: int = 0) -> Context:
    if device not in _default_ctx:
        _default_ctx[device] = Context(device)
    return _default_ctx[device]


def release_default_context(device: int = 0) -> None:
    """Destroy the default context of a device and with it the workspaces it keeps
    between calls (the next call without a context starts a new one)."""
    ctx = _default_ctx.pop(device, None)
    if ctx is not None:
        ctx.close()


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, torch.Tensor):
        return ctypes.c_void_p(x.data_ptr())
    return ctypes.c_void_p(x.ctypes.data)


def compute_batch(structures, params: MethodParams, species_table, *, forces=True, ctx: Context = None,
                  stream=None, want_alpha=False, want_dv=False, want_spectrum=False, static_scratch=False):
    """Energies and forces of several structures in one set of launches.

    ``structures``: list of dicts with keys pos (N,3), species (N,), v_ratio (N,),
    cell (3,3) or None, pbc (3,), cutoffs {r_scs, r_nbr, r_mbd1, r_mbd2[, r_2b1, r_2b2]} and
    optionally e_weight (N,).  Arrays are either all CUDA tensors (float64/int32,
    results are CUDA tensors, work on the current or given stream) or all host
    numpy arrays (results are numpy arrays).
    Returns a list of dicts {energies, forces?, alpha_scs0?, dE_dv?, spectrum?} (dE_dv: the
    exact derivative of sum_k w_k E_k with respect to the Hirshfeld-volume ratios, eV;
    spectrum: (N, n_freq, 2) Lanczos bounds of the spectrum of G~ per atom and node).
    ``static_scratch`` calls the entry point that allocates no device memory (its
    workspace is the library's static device array; small structures only).
    """
    device_mode = isinstance(structures[0]["pos"], torch.Tensor) and structures[0]["pos"].is_cuda
    if ctx is None:
        dev = structures[0]["pos"].device.index if device_mode else 0
        ctx = default_context(dev or 0)
    p, keep = params.to_c()
    sp, n_sp = species_array(species_table)
    descs = (C.StructureDesc * len(structures))()
    outs = []
    for i, s in enumerate(structures):
        if device_mode:
            pos = s["pos"].contiguous()
            spc = s["species"].to(torch.int32).contiguous()
            nu = s["v_ratio"].contiguous()
            w = s.get("e_weight")
            w = None if w is None else w.contiguous()
            e = torch.empty(pos.shape[0], dtype=torch.float64, device=pos.device)
            f = torch.empty_like(pos) if forces else None
            a = torch.empty_like(e) if want_alpha else None
            dv = torch.empty_like(e) if want_dv else None
            spec = torch.empty((pos.shape[0], p.n_freq, 2), dtype=torch.float64, device=pos.device) \
                if want_spectrum else None
        else:
            pos = np.ascontiguousarray(s["pos"], dtype=np.float64)
            spc = np.ascontiguousarray(s["species"], dtype=np.int32)
            nu = np.ascontiguousarray(s["v_ratio"], dtype=np.float64)
            w = s.get("e_weight")
            w = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
            e = np.empty(pos.shape[0])
            f = np.empty_like(pos) if forces else None
            a = np.empty_like(e) if want_alpha else None
            dv = np.empty_like(e) if want_dv else None
            spec = np.empty((pos.shape[0], p.n_freq, 2)) if want_spectrum else None
        cell = s.get("cell")
        cell_np = None if cell is None else np.ascontiguousarray(
            cell.detach().cpu().numpy() if isinstance(cell, torch.Tensor) else cell, dtype=np.float64)
        pbc = s.get("pbc", (0, 0, 0))
        pbc = [int(bool(x)) for x in (pbc.tolist() if hasattr(pbc, "tolist") else pbc)]
        cut = s["cutoffs"]
        keep.extend([pos, spc, nu, w, e, f, a, dv, spec, cell_np])
        descs[i] = C.StructureDesc(
            int(pos.shape[0]), _ptr(pos), _ptr(spc), _ptr(nu),
            cell_np.ctypes.data_as(C._dp) if cell_np is not None else None,
            (ctypes.c_int32 * 3)(*pbc), float(cut["r_scs"]), float(cut["r_nbr"]),
            float(cut["r_mbd1"]), float(cut["r_mbd2"]), float(cut.get("r_2b1") or 0.0),
            float(cut.get("r_2b2") or 0.0), _ptr(w), _ptr(e), _ptr(f), _ptr(a), _ptr(dv),
            _ptr(spec))
        outs.append({"energies": e, "forces": f, "alpha_scs0": a, "dE_dv": dv, "spectrum": spec})
    if device_mode:
        if stream is None:
            stream = torch.cuda.current_stream(structures[0]["pos"].device)
        hs = ctypes.c_void_p(stream.cuda_stream)
        mem = C.LMBD_DEVICE
    else:
        hs = None
        mem = C.LMBD_HOST
    entry = ctx.lib.lmbd_compute_batch_static if static_scratch else ctx.lib.lmbd_compute_batch
    st = entry(ctx.handle, ctypes.byref(p), n_sp, sp, len(structures), descs, mem, hs)
    if st != 0:
        raise C.LmbdError(st, ctx.last_error())
    return outs


def compute(pos, species, v_ratio, *, cutoffs, params: MethodParams, species_table, cell=None,
            pbc=None, e_weight=None, forces=True, ctx: Context = None, stream=None, want_alpha=False,
            want_dv=False, want_spectrum=False):
    """Per-atom energies (eV) and forces (eV/A) of one structure."""
    if pbc is None:
        pbc = (1, 1, 1) if cell is not None else (0, 0, 0)
    s = dict(pos=pos, species=species, v_ratio=v_ratio, cell=cell, pbc=pbc, cutoffs=cutoffs,
             e_weight=e_weight)
    return compute_batch([s], params, species_table, forces=forces, ctx=ctx, stream=stream,
                         want_alpha=want_alpha, want_dv=want_dv, want_spectrum=want_spectrum)[0]


def _host_desc(s, forces, keep):
    """StructureDesc of a structure dict with host (numpy) arrays; outputs allocated here."""
    pos = np.ascontiguousarray(s["pos"], dtype=np.float64)
    spc = np.ascontiguousarray(s["species"], dtype=np.int32)
    nu = np.ascontiguousarray(s["v_ratio"], dtype=np.float64)
    w = s.get("e_weight")
    w = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
    cell = s.get("cell")
    cell_np = None if cell is None else np.ascontiguousarray(cell, dtype=np.float64)
    pbc = s.get("pbc")
    if pbc is None:
        pbc = (1, 1, 1) if cell is not None else (0, 0, 0)
    pbc = [int(bool(x)) for x in (pbc.tolist() if hasattr(pbc, "tolist") else pbc)]
    e = np.empty(pos.shape[0])
    f = np.empty_like(pos) if forces else None
    a = np.empty(pos.shape[0])
    keep.extend([pos, spc, nu, w, cell_np, e, f, a])
    cut = s["cutoffs"]
    d = C.StructureDesc(
        int(pos.shape[0]), _ptr(pos), _ptr(spc), _ptr(nu),
        cell_np.ctypes.data_as(C._dp) if cell_np is not None else None,
        (ctypes.c_int32 * 3)(*pbc), float(cut["r_scs"]), float(cut["r_nbr"]),
        float(cut["r_mbd1"]), float(cut["r_mbd2"]), float(cut.get("r_2b1") or 0.0),
            float(cut.get("r_2b2") or 0.0), _ptr(w), _ptr(e), _ptr(f), _ptr(a), None)
    return d, {"energies": e, "forces": f, "alpha_scs0": a}


def estimate_footprint(structures, params: MethodParams, forces=True) -> int:
    """Exact device bytes of one call on these (host-array) structures."""
    p, keep = params.to_c()
    descs = (C.StructureDesc * len(structures))()
    for i, s in enumerate(structures):
        descs[i], _ = _host_desc(s, forces, keep)
    out = ctypes.c_size_t(0)
    st = C.lib().lmbd_estimate_footprint(ctypes.byref(p), len(structures), descs, ctypes.byref(out))
    if st != 0:
        raise C.LmbdError(st)
    return int(out.value)


def _info_dict(info):
    return {"done": bool(info.done), "status": C.STATUS.get(info.status, str(info.status)),
            "t_submit": info.t_submit, "t_start": info.t_start, "t_end": info.t_end,
            "footprint": int(info.footprint), "batch": int(info.batch),
            "batch_requests": int(info.batch_requests), "slot": int(info.slot),
            "detail": info.detail.decode(errors="replace")}


class Server:
    """Continuous-batching server (one device pool, ``n_slots`` concurrent batches).

    ``submit`` queues one structure (host arrays, copied here and kept alive
    until the request is released) and returns a ticket; ``wait``/``poll``
    return the outputs with the request's timing (seconds since the server was
    created) and the batch that ran it.
    """

    def __init__(self, params: MethodParams, species_table, *, device=0, n_slots=2, memory_budget=0,
                 max_batch_atoms=0, max_batch_requests=0):
        self.lib = C.lib()
        p, self._keep = params.to_c()
        sp, n_sp = species_array(species_table)
        cfg = C.ServerConfig(int(device), int(n_slots), ctypes.c_size_t(int(memory_budget)),
                             int(max_batch_atoms), int(max_batch_requests))
        h = ctypes.c_void_p()
        st = self.lib.lmbd_server_create(ctypes.byref(cfg), ctypes.byref(p), n_sp, sp, ctypes.byref(h))
        if st != 0:
            raise C.LmbdError(st, "lmbd_server_create")
        self.handle = h
        self._live = {}

    def submit(self, structure: dict, forces=True) -> int:
        keep = []
        desc, outs = _host_desc(structure, forces, keep)
        t = ctypes.c_uint64(0)
        st = self.lib.lmbd_submit(self.handle, ctypes.byref(desc), ctypes.byref(t))
        if st != 0:
            raise C.LmbdError(st, "lmbd_submit")
        self._live[t.value] = (keep, outs)
        return int(t.value)

    def _result(self, ticket, info):
        d = _info_dict(info)
        if info.done:
            d.update(self._live[ticket][1])
        return d

    def poll(self, ticket: int) -> dict:
        info = C.RequestInfo()
        st = self.lib.lmbd_poll(self.handle, ctypes.c_uint64(ticket), ctypes.byref(info))
        if st != 0:
            raise C.LmbdError(st, "lmbd_poll")
        return self._result(ticket, info)

    def wait(self, ticket: int) -> dict:
        info = C.RequestInfo()
        st = self.lib.lmbd_wait(self.handle, ctypes.c_uint64(ticket), ctypes.byref(info))
        if st != 0:
            raise C.LmbdError(st, "lmbd_wait")
        return self._result(ticket, info)

    def release(self, ticket: int):
        st = self.lib.lmbd_release(self.handle, ctypes.c_uint64(ticket))
        if st != 0:
            raise C.LmbdError(st, "lmbd_release")
        self._live.pop(ticket, None)

    def stats(self) -> dict:
        s = C.ServerStats()
        st = self.lib.lmbd_server_get_stats(self.handle, ctypes.byref(s))
        if st != 0:
            raise C.LmbdError(st)
        return {k: getattr(s, k) for k, _ in C.ServerStats._fields_}

    def close(self):
        if getattr(self, "handle", None):
            self.lib.lmbd_server_destroy(self.handle)
            self.handle = None
            self._live.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class LMBDEnergy(torch.autograd.Function):
    """Per-atom lMBD energies as a differentiable function of positions.

    backward() runs the library once more with the incoming gradient as the
    adjoint seeds w_k and returns -forces = d(sum_k w_k E_k)/dR and, when the
    volume ratios require a gradient, dE_dv = d(sum_k w_k E_k)/d nu.
    """

    @staticmethod
    def forward(ctx, pos, species, v_ratio, cell, cutoffs, params, species_table):
        out = compute(pos.detach(), species, v_ratio.detach(), cutoffs=cutoffs, params=params,
                      species_table=species_table, cell=cell, forces=False)
        ctx.save_for_backward(pos, species, v_ratio)
        ctx.extra = (cell, cutoffs, params, species_table)
        return out["energies"]

    @staticmethod
    def backward(ctx, grad_e):
        pos, species, v_ratio = ctx.saved_tensors
        cell, cutoffs, params, species_table = ctx.extra
        want_dv = ctx.needs_input_grad[2]
        out = compute(pos.detach(), species, v_ratio.detach(), cutoffs=cutoffs, params=params,
                      species_table=species_table, cell=cell, e_weight=grad_e.contiguous(), forces=True,
                      want_dv=want_dv)
        return -out["forces"], None, out["dE_dv"] if want_dv else None, None, None, None, None
