"""Helpers shared by the GPU parity tests: oracle state <-> C-ABI component arrays."""
import numpy as np
import pytest

from oracle import components, lattice, init_mv

gpu = pytest.mark.gpu


def lattice_or_skip():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_2009_02044_amd as pkg
    return pkg


def to_comp(st):
    return (components.links_to_comp(st.U), components.alg_to_comp(st.E),
            components.alg_to_comp(st.rhoA), components.alg_to_comp(st.rhoB))


def from_comp(d, nc, dims, params):
    U = components.comp_to_links(d["U"], nc, dims)
    E = components.comp_to_alg(d["E"], nc, dims, lead=(3,))
    rA = components.comp_to_alg(d["rhoA"], nc, dims)
    rB = components.comp_to_alg(d["rhoB"], nc, dims)
    return lattice.State(U, E, rA, rB, d["step"], params)


def field_err(got, ref):
    """max |got - ref| / max(|ref|, RMS(ref)) over the whole field (elementwise)."""
    ref = np.asarray(ref)
    rms = np.sqrt(np.mean(ref ** 2)) if ref.size else 0.0
    den = np.maximum(np.abs(ref), rms)
    den = np.where(den > 0, den, 1.0)
    return float(np.max(np.abs(np.asarray(got) - ref) / den)) if ref.size else 0.0


def state_errs(gpu_state, st):
    U, E, rA, rB = to_comp(st)
    return {"U": field_err(gpu_state["U"], U), "E": field_err(gpu_state["E"], E),
            "rhoA": field_err(gpu_state["rhoA"], rA), "rhoB": field_err(gpu_state["rhoB"], rB)}


def mv_setup(w):
    p = lattice.Params(nc=w.nc, a_T=w.a_T, a_L=w.a_L, dt=w.dt)
    mv = init_mv.MVParams(m_ir=w.m_ir, uv_cut=w.uv_cut, sigma=w.sigma, zA=w.zA, zB=w.zB)
    return p, mv


def new_lattice(pkg, w, fp=64, **kw):
    return pkg.Lattice(nc=w.nc, nz=w.nz, nt=w.nt, a_T=w.a_T, a_L=w.a_L, dt=w.dt, fp=fp, **kw)
