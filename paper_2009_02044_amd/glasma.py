"""Python front end of the HIP library: torch owns the device memory and the stream,
every computation runs in libglasma.so.  Names follow the C-ABI (include/glasma.h)."""
import ctypes as C
import numpy as np
import torch

from . import _lib
from ._lib import lib, check, dptr


def _device(device):
    """torch.device with an explicit index (tensors report cuda:k)."""
    d = torch.device(device)
    if d.type == "cuda" and d.index is None:
        d = torch.device("cuda", torch.cuda.current_device())
    return d


class Lattice:
    """One event: SU(nc) links, E field and the two nuclei's CPIC charges on an
    nz x nt x nt lattice held in caller-owned (torch) device buffers."""

    def __init__(self, nc, nz, nt, a_T=4.0, a_L=1.0, dt=0.5, fp=64, scheme=0,
                 reunit_every=0, max_iter=50, tol=0.0, device="cuda", _ctx=None, _stream=None):
        if _ctx is not None:      # a view of an event owned by a Batch
            self.params = _lib.Params(nc, nz, nt, a_T, a_L, dt, fp, scheme, reunit_every, max_iter, tol)
            self.stream = _stream
            self.ctx = _ctx
            self._owned = False
            self.device = _device(device)
            self._set_dims(nc, nz, nt, fp)
            return
        if not torch.cuda.is_available():
            raise RuntimeError("the HIP library needs a GPU; no device is visible")
        self.params = _lib.Params(nc, nz, nt, a_T, a_L, dt, fp, scheme, reunit_every, max_iter, tol)
        sizes = (C.c_size_t * 6)()
        check(lib.glasma_layout(C.byref(self.params), sizes))
        self.sizes = list(sizes)
        self.device = _device(device)
        self._bufs = [torch.empty(max(int(s), 1), dtype=torch.uint8, device=self.device) for s in self.sizes]
        b = _lib.Buffers(*[t.data_ptr() for t in self._bufs])
        self.stream = torch.cuda.current_stream(self.device)
        self.ctx = C.c_void_p()
        check(lib.glasma_create(C.byref(self.params), C.byref(b), C.c_void_p(self.stream.cuda_stream),
                                C.byref(self.ctx)))
        self._owned = True
        self._set_dims(nc, nz, nt, fp)

    def _set_dims(self, nc, nz, nt, fp):
        self.nc, self.nz, self.nt, self.fp = nc, nz, nt, fp
        self.ng = nc * nc - 1
        self.r = 4 if nc == 2 else 18
        self.V = nz * nt * nt
        self.real = torch.float64 if fp == 64 else torch.float32

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if getattr(self, "_owned", False) and ctx is not None and ctx.value:
            lib.glasma_destroy(ctx)
            self.ctx = None

    def _chk(self, rc):
        return check(rc, self.ctx)

    # -- state ------------------------------------------------------------------
    def init_state(self, U, E, rhoA, rhoB, step0=0):
        """Host float64 arrays in the C-ABI layout: U (3, r_U, V), E (3, n_g, V), rho (n_g, V)."""
        arrs = [np.ascontiguousarray(x, dtype=np.float64) for x in (U, E, rhoA, rhoB)]
        self._chk(lib.glasma_init_state(self.ctx, *[dptr(a) for a in arrs], int(step0)))

    def init_mv(self, rhoT_A, rhoT_B, m_ir=0.2, uv_cut=0.0, sigma=4.0, zA=None, zB=None):
        """MV nuclei from transverse charges (n_g, nt, nt) per nucleus, or (ns, n_g, nt, nt)
        for ns colour sheets along the beam axis (glasma_init_mv_sheets)."""
        zA = 0.75 * self.nz * self.params.a_L if zA is None else zA
        zB = 0.25 * self.nz * self.params.a_L if zB is None else zB
        mv = _lib.MV(m_ir, uv_cut, sigma, zA, zB)
        a = np.ascontiguousarray(rhoT_A, dtype=np.float64)
        b = np.ascontiguousarray(rhoT_B, dtype=np.float64)
        if a.shape != b.shape or a.ndim not in (3, 4):
            raise ValueError("rhoT_A and rhoT_B must both be (n_g, nt, nt) or (ns, n_g, nt, nt)")
        if a.ndim == 3:
            self._chk(lib.glasma_init_mv(self.ctx, C.byref(mv), dptr(a), dptr(b)))
        else:
            self._chk(lib.glasma_init_mv_sheets(self.ctx, C.byref(mv), int(a.shape[0]), dptr(a), dptr(b)))

    def step(self, n=1):
        self._chk(lib.glasma_step(self.ctx, int(n)))

    def reunitarize(self):
        self._chk(lib.glasma_reunitarize(self.ctx))

    @property
    def last_iterations(self):
        """Fixed-point iterations of the last semi-implicit step."""
        n = C.c_int32()
        self._chk(lib.glasma_last_iterations(self.ctx, C.byref(n)))
        return n.value

    @property
    def step_count(self):
        s = C.c_int64()
        self._chk(lib.glasma_get_step(self.ctx, C.byref(s)))
        return s.value

    def get_state(self):
        U = np.empty((3, self.r, self.V))
        E = np.empty((3, self.ng, self.V))
        rA = np.empty((self.ng, self.V))
        rB = np.empty((self.ng, self.V))
        s = C.c_int64()
        self._chk(lib.glasma_get_state(self.ctx, dptr(U), dptr(E), dptr(rA), dptr(rB), C.byref(s)))
        return {"U": U, "E": E, "rhoA": rA, "rhoB": rB, "step": s.value}

    # -- derived quantities -----------------------------------------------------
    def deposit_current(self):
        j = torch.empty(3 * self.ng * self.V, dtype=self.real, device=self.device)
        self._chk(lib.glasma_deposit_current(self.ctx, C.c_void_p(j.data_ptr())))
        return j

    def obs_buffer(self):
        return torch.empty(4 * self.nz + _lib.OBS_NSCALARS, dtype=torch.float64, device=self.device)

    def observe(self, out):
        """Asynchronous: write slices + scalars into the float64 device tensor `out`."""
        self._chk(lib.glasma_observe(self.ctx, C.c_void_p(out.data_ptr())))

    def observe_noalloc(self, out):
        """As observe(), with the partial sums in the library's static device array
        (glasma_observe_noalloc: allocates nothing; leapfrog; lattices up to its limit)."""
        self._chk(lib.glasma_observe_noalloc(self.ctx, C.c_void_p(out.data_ptr())))

    def step_observe(self, n, out):
        """n >= 1 steps; `out` (an obs_buffer()) receives the observables of the state the
        last step starts from (glasma_step_observe).  Asynchronous."""
        self._chk(lib.glasma_step_observe(self.ctx, int(n), C.c_void_p(out.data_ptr())))

    def rest_frame(self, obs):
        """Local rest frame of every layer from an observe() buffer (glasma_rest_frame):
        device float64 tensor (2, nz) = [eps_loc, v]."""
        out = torch.empty(2, self.nz, dtype=torch.float64, device=self.device)
        self._chk(lib.glasma_rest_frame(self.ctx, C.c_void_p(obs.data_ptr()), C.c_void_p(out.data_ptr())))
        return out

    def observables(self):
        t = np.empty((4, self.nz))
        vals = [C.c_double() for _ in range(4)]
        self._chk(lib.glasma_observables(self.ctx, dptr(t), *[C.byref(v) for v in vals]))
        return {"tmunu_z": t, "gauss_rel": vals[0].value, "gauss_max": vals[1].value,
                "energy": vals[2].value, "unitarity": vals[3].value}

    # -- device state transfer (plain double layout of the C-ABI) -------------
    def _dev(self, t, shape, name):
        if t is None:
            return None
        if t.dtype != torch.float64 or t.device != self.device or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float64 tensor on {self.device}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
        return C.c_void_p(t.data_ptr())

    def set_state_device(self, U, E, rhoA, rhoB, ampA=None, ampB=None, step0=0):
        """Device float64 tensors U (3, r_U, V), E (3, n_g, V), rho (n_g, V); amp (V,) scales
        the charges of each cell."""
        self._chk(lib.glasma_set_state_device(
            self.ctx, self._dev(U, (3, self.r, self.V), "U"), self._dev(E, (3, self.ng, self.V), "E"),
            self._dev(rhoA, (self.ng, self.V), "rhoA"), self._dev(rhoB, (self.ng, self.V), "rhoB"),
            self._dev(ampA, (self.V,), "ampA"), self._dev(ampB, (self.V,), "ampB"), int(step0)))

    def get_state_device(self):
        f = dict(dtype=torch.float64, device=self.device)
        out = {"U": torch.empty(3, self.r, self.V, **f), "E": torch.empty(3, self.ng, self.V, **f),
               "rhoA": torch.empty(self.ng, self.V, **f), "rhoB": torch.empty(self.ng, self.V, **f)}
        self._chk(lib.glasma_get_state_device(self.ctx, *[C.c_void_p(out[k].data_ptr())
                                                          for k in ("U", "E", "rhoA", "rhoB")]))
        return out

    # -- differentiation form ----------------------------------------------------
    def slab_energy(self, z0, z1):
        """Electric + magnetic energy of layers [z0, z1) of the current state (glasma_slab_energy)."""
        v = C.c_double()
        self._chk(lib.glasma_slab_energy(self.ctx, int(z0), int(z1), C.byref(v)))
        return v.value

    def adjoint_work(self, steps, ckpt_every):
        n = C.c_size_t()
        check(lib.glasma_adjoint_layout(C.byref(self.params), int(steps), int(ckpt_every), C.byref(n)))
        return torch.empty(max(n.value, 1), dtype=torch.uint8, device=self.device)

    def adjoint_forward(self, steps, ckpt_every, work):
        self._chk(lib.glasma_adjoint_forward(self.ctx, int(steps), int(ckpt_every), C.c_void_p(work.data_ptr()),
                                             work.numel()))

    def adjoint_backward(self, z0, z1, work, scale=1.0, baseA=None, baseB=None):
        """Gradients of scale * L with respect to the state before the last adjoint_forward:
        dE0 (3, n_g, V), drhoA0 / drhoB0 (n_g, V), dampA / dampB (V,); L (unscaled)."""
        f = dict(dtype=torch.float64, device=self.device)
        out = {"dE0": torch.empty(3, self.ng, self.V, **f), "drhoA0": torch.empty(self.ng, self.V, **f),
               "drhoB0": torch.empty(self.ng, self.V, **f), "dampA": torch.empty(self.V, **f),
               "dampB": torch.empty(self.V, **f)}
        L = C.c_double()
        self._chk(lib.glasma_adjoint_backward(
            self.ctx, int(z0), int(z1), float(scale), C.c_void_p(work.data_ptr()), work.numel(),
            self._dev(baseA, (self.ng, self.V), "baseA"), self._dev(baseB, (self.ng, self.V), "baseB"),
            C.byref(L), *[C.c_void_p(out[k].data_ptr()) for k in ("dE0", "drhoA0", "drhoB0", "dampA", "dampB")]))
        out["L"] = L.value
        return out

    def adjoint_backward_cotangent(self, work, lamU=None, ebarE=None, rbarA=None, rbarB=None, baseA=None,
                                   baseB=None):
        """Gradients of a general loss of the final state of the last adjoint_forward, given
        its cotangent (device float64 tensors, None = 0): lamU, ebarE (3, n_g, V); rbarA,
        rbarB (n_g, V).  Returns dU0, dE0 (3, n_g, V), drhoA0, drhoB0 (n_g, V), dampA, dampB (V,)."""
        f = dict(dtype=torch.float64, device=self.device)
        out = {"dU0": torch.empty(3, self.ng, self.V, **f), "dE0": torch.empty(3, self.ng, self.V, **f),
               "drhoA0": torch.empty(self.ng, self.V, **f), "drhoB0": torch.empty(self.ng, self.V, **f),
               "dampA": torch.empty(self.V, **f), "dampB": torch.empty(self.V, **f)}
        self._chk(lib.glasma_adjoint_backward_cotangent(
            self.ctx, C.c_void_p(work.data_ptr()), work.numel(),
            self._dev(lamU, (3, self.ng, self.V), "lamU"), self._dev(ebarE, (3, self.ng, self.V), "ebarE"),
            self._dev(rbarA, (self.ng, self.V), "rbarA"), self._dev(rbarB, (self.ng, self.V), "rbarB"),
            self._dev(baseA, (self.ng, self.V), "baseA"), self._dev(baseB, (self.ng, self.V), "baseB"),
            *[C.c_void_p(out[k].data_ptr()) for k in ("dU0", "dE0", "drhoA0", "drhoB0", "dampA", "dampB")]))
        return out

    @staticmethod
    def unpack_obs(buf, nz):
        h = buf.detach().cpu().numpy()
        s = h[4 * nz:]
        out = {k: float(s[v]) for k, v in _lib.OBS.items()}
        out["tmunu_z"] = h[:4 * nz].reshape(4, nz)
        return out


class Batch:
    """Many events of different sizes in one device pool, advanced together
    (glasma_batch_*).  The batch runs on its own (non-default) stream so that steps can
    be captured in a HIP graph; every event is reachable as a Lattice view."""

    def __init__(self, nc, shapes, a_T=4.0, a_L=1.0, dt=0.5, fp=32, reunit_every=8, device="cuda"):
        if not torch.cuda.is_available():
            raise RuntimeError("the HIP library needs a GPU; no device is visible")
        from ._lib import check_batch
        self._check = check_batch
        self.params = _lib.Params(nc, 0, 0, a_T, a_L, dt, fp, 0, reunit_every, 1, 0.0)
        n = len(shapes)
        self.nz = (C.c_int32 * n)(*[int(s[0]) for s in shapes])
        self.nt = (C.c_int32 * n)(*[int(s[1]) for s in shapes])
        size = C.c_size_t()
        check_batch(lib.glasma_batch_layout(C.byref(self.params), n, self.nz, self.nt, C.byref(size)))
        self.device = _device(device)
        self.pool = torch.empty(size.value, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.Stream(self.device)
        self.b = C.c_void_p()
        check_batch(lib.glasma_batch_create(C.byref(self.params), n, self.nz, self.nt,
                                            C.c_void_p(self.pool.data_ptr()),
                                            C.c_void_p(self.stream.cuda_stream), C.byref(self.b)))
        self.events = []
        for e in range(n):
            ctx = C.c_void_p()
            check_batch(lib.glasma_batch_event(self.b, e, C.byref(ctx)), self.b)
            self.events.append(Lattice(nc, shapes[e][0], shapes[e][1], a_T, a_L, dt, fp, 0, reunit_every,
                                       1, 0.0, device, _ctx=ctx, _stream=self.stream))
        self.sites = sum(int(s[0]) * int(s[1]) ** 2 for s in shapes)

    def __del__(self):
        b = getattr(self, "b", None)
        if b is not None and b.value:
            lib.glasma_batch_destroy(b)
            self.b = None

    def run(self, steps, graph_chunk=16):
        self._check(lib.glasma_batch_run(self.b, int(steps), int(graph_chunk)), self.b)

    def classes(self):
        """N_z classes of the events: list of (N_z, number of events), ascending."""
        n = len(self.events)
        k = C.c_int32()
        nz = (C.c_int32 * n)()
        cnt = (C.c_int32 * n)()
        self._check(lib.glasma_batch_classes(self.b, C.byref(k), nz, cnt), self.b)
        return [(int(nz[i]), int(cnt[i])) for i in range(k.value)]

    def observe(self, n_grid, per_event=False):
        """Event-averaged T^{mu nu}(z) (glasma_batch_observe), device float64 tensors:
        {"class": {N_z: (4, N_z)}, "grid": (4, n_grid)} and, with per_event, the events'
        observables buffers (one flat tensor, events in order).  Asynchronous."""
        cls = self.classes()
        f = dict(dtype=torch.float64, device=self.device)
        cbuf = torch.empty(sum(4 * nz for nz, _ in cls), **f)
        gbuf = torch.empty(4 * int(n_grid), **f)
        pe = torch.empty(sum(4 * lat.nz + _lib.OBS_NSCALARS for lat in self.events), **f) if per_event else None
        self._check(lib.glasma_batch_observe(self.b, int(n_grid), C.c_void_p(cbuf.data_ptr()),
                                             C.c_void_p(gbuf.data_ptr()),
                                             C.c_void_p(pe.data_ptr()) if pe is not None else None), self.b)
        out, o = {}, 0
        for nz, _ in cls:
            out[nz] = cbuf[o:o + 4 * nz].view(4, nz)
            o += 4 * nz
        r = {"class": out, "grid": gbuf.view(4, int(n_grid))}
        if per_event:
            r["per_event"] = pe
        return r

    def set_tiling(self, sites_per_item, grid):
        self._check(lib.glasma_batch_set_tiling(self.b, int(sites_per_item), int(grid)), self.b)

    def autotune(self, steps=2):
        import json
        buf = C.create_string_buffer(8192)
        self._check(lib.glasma_batch_autotune(self.b, int(steps), buf, 8192), self.b)
        return json.loads(buf.value.decode())


class SlabEnergy(torch.autograd.Function):
    """L(E0, ampA, ampB): energy of layers [z0, z1) after `steps` leapfrog steps of `lat`
    from the state (U0, E0, ampA * rhoA, ampB * rhoB) at step 0, with U0 held fixed.
    Forward: glasma_adjoint_forward (checkpoint every ckpt_every steps) and
    glasma_slab_energy; backward: glasma_adjoint_backward.  E0 (3, n_g, V), amp (V,),
    U0 (3, r_U, V) and the base charges (n_g, V) are float64 device tensors."""

    @staticmethod
    def forward(ctx, E0, ampA, ampB, lat, U0, rhoA, rhoB, steps, ckpt_every, z0, z1):
        lat.set_state_device(U0, E0.contiguous(), rhoA, rhoB, ampA.contiguous(), ampB.contiguous(), 0)
        work = lat.adjoint_work(steps, ckpt_every)
        lat.adjoint_forward(steps, ckpt_every, work)
        L = lat.slab_energy(z0, z1)
        ctx.lat, ctx.work, ctx.slab = lat, work, (z0, z1)
        ctx.save_for_backward(rhoA, rhoB)
        return torch.tensor(L, dtype=torch.float64, device=E0.device)

    @staticmethod
    def backward(ctx, gL):
        rhoA, rhoB = ctx.saved_tensors
        g = ctx.lat.adjoint_backward(ctx.slab[0], ctx.slab[1], ctx.work, scale=float(gL), baseA=rhoA, baseB=rhoB)
        return (g["dE0"], g["dampA"], g["dampB"]) + (None,) * 8


def host_group_op(nc, fp, op, inp, n_out_per_item):
    """Evaluate the device group algebra on the host (see glasma_host_group_op)."""
    inp = np.ascontiguousarray(inp, dtype=np.float64)
    n = inp.shape[0]
    out = np.empty((n, n_out_per_item))
    check(lib.glasma_host_group_op(nc, fp, op, n, dptr(inp), dptr(out)))
    return out


def boost_invariant_fields(nc, nt, rhoT_A, rhoT_B, a_T=4.0, m_ir=0.2, uv_cut=0.0, device="cuda"):
    """Boost-invariant Glasma at tau = 0+ of two nuclei (glasma_bi_fields): E_z at the
    sites and B_z at the plaquette centres, each (n_g, nt, nt) float64 on the device, and
    the transverse means {"eps0", "EL2_half", "BL2_half"}.  rhoT_*: (n_g, nt, nt) or
    (ns, n_g, nt, nt) host charges, as for Lattice.init_mv."""
    if not torch.cuda.is_available():
        raise RuntimeError("the HIP library needs a GPU; no device is visible")
    a = np.ascontiguousarray(rhoT_A, dtype=np.float64)
    b = np.ascontiguousarray(rhoT_B, dtype=np.float64)
    if a.shape != b.shape or a.ndim not in (3, 4):
        raise ValueError("rhoT_A and rhoT_B must both be (n_g, nt, nt) or (ns, n_g, nt, nt)")
    ns = 1 if a.ndim == 3 else a.shape[0]
    ng = nc * nc - 1
    if a.shape[-3:] != (ng, nt, nt):
        raise ValueError(f"charges must end in ({ng}, {nt}, {nt})")
    params = _lib.Params(nc, 2, nt, a_T, 1.0, 0.5, 64, 0, 0, 50, 0.0)
    mv = _lib.MV(m_ir, uv_cut, 1.0, 0.0, 0.0)
    nbytes = C.c_size_t()
    check(lib.glasma_bi_work_bytes(C.byref(params), C.byref(nbytes)))
    dev = _device(device)
    work = torch.empty(int(nbytes.value), dtype=torch.uint8, device=dev)
    Ez = torch.empty((ng, nt, nt), dtype=torch.float64, device=dev)
    Bz = torch.empty_like(Ez)
    out = torch.empty(3, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    check(lib.glasma_bi_fields(C.byref(params), C.byref(mv), int(ns), dptr(a), dptr(b), C.c_void_p(work.data_ptr()),
                               C.c_void_p(Ez.data_ptr()), C.c_void_p(Bz.data_ptr()), C.c_void_p(out.data_ptr()),
                               C.c_void_p(stream.cuda_stream)))
    o = out.cpu().numpy()
    return {"Ez": Ez, "Bz": Bz, "eps0": float(o[0]), "EL2_half": float(o[1]), "BL2_half": float(o[2])}
