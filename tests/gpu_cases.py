"""Helpers shared by the GPU parity tests: build the same state in the HIP
library (through the C ABI) and in the FP64 oracle, and compare them."""
import numpy as np

PAIR = [(-1.0, 1.0), (1.0, 1.0)]


def sim(dims, n_x, rho0, maxp, dt=0.5, species=PAIR, fp64=False, tile=(4, 4, 4), **kw):
    from paper_1308_5892_amd import pic as P
    boxes = [{"n": tuple(dims), "n_x": n_x, "rho0": rho0, "max_particles": list(maxp), "tile": tile}]
    return P.Simulation(boxes, species, dt, fp64=fp64, track_ids=True, **kw)


def oracle_state(dims, n_x, rho0, dt=0.5, species=PAIR):
    from oracle import oracle as O
    return O.State(dims, dt, n_x, rho0, species)


def copy_to_oracle(s, st, box=0):
    """Load the GPU's particles and fields (ordered by id) into an oracle state."""
    e, b, _ = s.fields(box)
    st.e = e.copy()
    st.b = b.copy()
    st.x = np.zeros((0, 3))
    st.u = np.zeros((0, 3))
    st.species = np.zeros(0, dtype=np.int32)
    for sp in range(s.nsp):
        x, u, _ = s.particles(box, sp)
        st.add_particles(sp, x, u)


def wrap_delta(x, ref, dims):
    d = np.asarray(x) - np.asarray(ref)
    L = np.asarray(dims, dtype=float)
    return d - L * np.round(d / L)


def u_rel_err(u, ref, floor):
    """per-particle |du| / max(|u_ref|, floor)"""
    nu = np.maximum(np.linalg.norm(ref, axis=1), floor)
    return np.linalg.norm(np.asarray(u) - np.asarray(ref), axis=1) / nu


def random_fields(rng, n, amp_e, amp_b):
    return amp_e * rng.standard_normal(3 * n), amp_b * rng.standard_normal(3 * n)
