"""Helpers shared by the GPU tests: build one starting state from test inputs
(or from the oracle's own loader), round it to the library's storage format,
and hand the same values to the HIP library (through the C ABI) and to the FP64
oracle.  Nothing the HIP path computes ever becomes an oracle input."""
import numpy as np

PAIR = [(-1.0, 1.0), (1.0, 1.0)]


def sim(dims, n_x, rho0, maxp, dt=0.5, species=PAIR, fp64=False, tile=(4, 4, 4), **kw):
    from paper_1308_5892_amd import pic as P
    boxes = [{"n": tuple(dims), "n_x": n_x, "rho0": rho0, "max_particles": list(maxp), "tile": tile}]
    return P.Simulation(boxes, species, dt, fp64=fp64, track_ids=True, **kw)


def oracle_state(dims, n_x, rho0, dt=0.5, species=PAIR):
    from oracle import oracle as O
    return O.State(dims, dt, n_x, rho0, species)


def to_storage(x, u, dims, fp64):
    """The particle state as the library stores it: positions wrapped into the
    box as integer cell plus in-cell offset, the offset and the momentum in the
    form's precision (FP32 form: both rounded to nearest FP32; FP64 form: as
    given).  Values returned are exactly representable in that storage."""
    L = np.asarray(dims, dtype=float)
    x = np.mod(np.asarray(x, dtype=float).reshape(-1, 3), L)
    u = np.asarray(u, dtype=float).reshape(-1, 3)
    c = np.floor(x)
    d = x - c
    if not fp64:
        d = d.astype(np.float32).astype(np.float64)
        u = u.astype(np.float32).astype(np.float64)
    up = d >= 1.0                      # rounding reached the next cell
    d[up] = 0.0
    c[up] += 1.0
    c = np.mod(c, L)
    return c + d, u.copy()


def field_storage(f, fp64):
    f = np.asarray(f, dtype=float)
    return f.copy() if fp64 else f.astype(np.float32).astype(np.float64)


def start(s, st, parts, box=0, e=None, b=None, fp64=False):
    """Give the GPU context `s` and the oracle state `st` the same start:
    parts[sp] = (x, u) per species (rounded to storage here), ids 0..n-1 per
    species in the given order; optional e and b (rounded likewise)."""
    dims = st.dims
    if e is not None or b is not None:
        n = 3 * int(np.prod(dims))
        e = np.zeros(n) if e is None else field_storage(e, fp64)
        b = np.zeros(n) if b is None else field_storage(b, fp64)
        s.set_fields(box, e, b)
        st.e, st.b = e.copy(), b.copy()
    for sp, (x, u) in enumerate(parts):
        xs, us = to_storage(x, u, dims, fp64)
        s.set_particles(box, sp, xs, us, np.arange(len(xs)))
        st.add_particles(sp, xs, us)


def oracle_loaded(dims, dt, n_x, rho0, species, loads, b=None):
    """Particles of one or more pair loads drawn by the oracle's loader
    (Sect. 4.3, App. D) and integrated back by dt/2 in the fields e = 0 and b
    (App. A.3.1).  loads: dicts with seed, stream, npairs, A, B and optional
    profile keywords of oracle.load_pairs.  Returns [(x, u)] per species, pairs
    of all loads in load order (species 0 from A, species 1 from B)."""
    from oracle import oracle as O
    st = O.State(dims, dt, n_x, rho0, species)
    if b is not None:
        st.b = np.asarray(b, dtype=float).copy()
    xs, ua, ub = [], [], []
    for ld in loads:
        x, a, bb = O.load_pairs(dims, ld["seed"], ld["stream"], ld["npairs"], ld["A"], ld["B"],
                                **ld.get("prof", {}))
        xs.append(x)
        ua.append(a)
        ub.append(bb)
    x = np.concatenate(xs)
    st.add_particles(0, x, np.concatenate(ua))
    st.add_particles(1, x, np.concatenate(ub))
    st.backward_half()
    return [(st.x[st.species == sp], st.u[st.species == sp]) for sp in range(2)]


def oblique_mode(dims, m, dt, amp=1.0):
    """A vacuum eigenmode of the discrete Yee scheme (App. A.3.2) with mode
    numbers m: e at t = 0 and b at t = -dt/2, transverse in the discrete sense
    (e perpendicular to kappa = 2 sin(k/2)), so its discrete div e is zero."""
    E_POS = np.array([[0.5, 0, 0], [0, 0.5, 0], [0, 0, 0.5]])
    B_POS = np.array([[0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]])
    kv = 2 * np.pi * np.array(m) / np.array(dims)
    kap = 2 * np.sin(kv / 2)
    e_hat = np.cross(kap, [0.3, 1.0, 0.2])
    e_hat /= np.linalg.norm(e_hat)
    s = 0.5 * dt * np.linalg.norm(kap)
    om = 2 * np.arcsin(s) / dt
    b_hat = dt * np.cross(kap, e_hat) / (2 * s)
    i, j, k = np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")
    X = [a.transpose(2, 1, 0).reshape(-1).astype(float) for a in (i, j, k)]
    e = np.concatenate([e_hat[c] * np.cos(sum(kv[a] * (X[a] + E_POS[c][a]) for a in range(3))) for c in range(3)])
    b = np.concatenate([b_hat[c] * np.cos(sum(kv[a] * (X[a] + B_POS[c][a]) for a in range(3)) + om * dt / 2)
                        for c in range(3)])
    return amp * e, amp * b


def beam_loads(w):
    """Two counter-streaming pair beams along x (Sect. 3.2): each a load of
    co-located pairs drifting with gamma beta = +-sqrt(gamma^2 - 1)."""
    gb = float(np.sqrt(w["gamma"] ** 2 - 1.0))
    npairs = int(round(w["ppc_per_beam"] * np.prod(w["dims"])))
    return [dict(seed=w["seed"], stream=k, npairs=npairs, A={"theta": w["theta"], "gb": sgn * gb, "axis": 0},
                 B={"theta": w["theta"], "gb": sgn * gb, "axis": 0}) for k, sgn in ((0, 1.0), (1, -1.0))]


def harris_setup(w):
    """Periodic double Harris sheet (App. C): gradient along x, b along y,
    drifts along z with opposite signs in the two sheets, plus a uniform
    non-drifting background.  Parameters from the oracle's App. C relations;
    d_e = n_x cells at the peak density, so L = (L/d_e) n_x cells and
    b0 = omega_ce = (omega_ce/omega_pe) / n_x.  Returns (species, b, loads,
    GPU load arguments, harris field arguments)."""
    from oracle import oracle as O
    dims = w["dims"]
    Lx = dims[0]
    hp = O.harris_params(w["theta_e"], w["gu_e"], w["chi"], w["mass_ratio"])
    L = hp["L_over_de"] * w["n_x"]
    b0 = hp["wce_over_wpe"] / w["n_x"]
    te, ti = w["theta_e"], hp["theta_i"]
    gi = (2.0 * w["chi"] - 1.0) * w["gu_e"]           # Gamma_i U_i / c (opposite to the electrons)
    cells = int(np.prod(dims))
    centres = [Lx / 4.0, 3.0 * Lx / 4.0]
    hw = Lx / 4.0
    n_sheet = int(round(w["ppc"] * (cells / Lx) * 2 * L * np.tanh(hw / L)))
    loads, gpu = [], []
    for k, (c, sg) in enumerate(zip(centres, (1.0, -1.0))):
        A = {"theta": te, "gb": -sg * w["gu_e"], "axis": 2}
        B = {"theta": ti, "gb": sg * gi, "axis": 2}
        loads.append(dict(seed=w["seed"], stream=k, npairs=n_sheet, A=A, B=B,
                          prof=dict(profile=1, paxis=0, centre=c, L=L, halfw=hw)))
        gpu.append(((te, A["gb"], 2), (ti, B["gb"], 2), w["ppc"],
                    dict(seed=w["seed"], stream=k, profile=1, profile_axis=0, centre=c, thickness=L,
                         half_width=hw)))
    nbg = int(round(w["background"] * w["ppc"] * cells))
    loads.append(dict(seed=w["seed"], stream=2, npairs=nbg, A={"theta": te, "gb": 0.0, "axis": 2},
                      B={"theta": ti, "gb": 0.0, "axis": 2}))
    gpu.append(((te, 0.0, 2), (ti, 0.0, 2), w["background"] * w["ppc"], dict(seed=w["seed"], stream=2)))
    n = cells
    i = np.arange(n) % Lx
    b = np.zeros(3 * n)
    b[n:2 * n] = b0 * (np.tanh((i + 0.5 - centres[0]) / L) - np.tanh((i + 0.5 - centres[1]) / L) - 1.0)
    species = [(-1.0, 1.0), (1.0, w["mass_ratio"])]
    return species, b, loads, gpu, (0, 1, b0, L, centres)


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
