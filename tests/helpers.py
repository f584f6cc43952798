"""Shared plumbing of the GPU parity tests: run the same seeded workload
through the HIP library (via its C ABI) and through the FP64 oracle."""
import math

import numpy as np

import oracle as o
import workloads as wl


def weights(dim):
    _, w = o.lattice(dim)
    return w


def gpu_solver(params_list, nodes_list=None, tris_list=None, storage=0):
    from paper_2503_20605_amd import Solver, params_from
    P = [params_from(p) for p in params_list]
    s = Solver(P, nodes_list, tris_list, storage=storage)
    for d, p in enumerate(params_list):
        lam = float(getattr(p, "lam", 1.0))
        if lam != 1.0:
            s.set_viscosity_ratio(d, lam)
        mu_s = float(getattr(p, "shear", 0.0))
        if mu_s != 0.0:
            s.set_membrane_shear(d, mu_s)
        beta = float(getattr(p, "respace", 0.0))
        if beta != 0.0:
            s.set_node_respacing(d, beta)
    return s


def gpu_run(p, q0, steps, tris=None, storage=0, f0dev=None, F_fixed=None, graph_steps=None,
            shape=None):
    """Run `steps` steps of one droplet on the GPU; returns a dict like
    oracle.run (numpy, float64) plus the solver."""
    s = gpu_solver([p], None if q0 is None else [q0], None if tris is None else [tris], storage)
    if graph_steps is not None:
        s.set_graph_steps(graph_steps)
    if shape is not None:
        s.set_lb_variant(shape)
    if f0dev is not None:
        s.write_populations(0, f0dev)
    if F_fixed is not None:
        s.set_force_field(0, F_fixed)
    s.step(steps)
    return collect(s, 0, p.dim)


def collect(s, d, dim):
    rho, U, F = s.read_fields(d)
    fdev = s.read_populations(d).cpu().numpy()
    out = dict(solver=s, rho=rho.cpu().numpy().astype(np.float64),
               U=U.cpu().numpy().astype(np.float64), F=F.cpu().numpy().astype(np.float64),
               fdev=fdev)
    if s.n_nodes[d] > 0:
        q, v, phi = s.read_nodes(d)
        out.update(q=q, qdot=v.astype(np.float64), phi=phi.astype(np.float64))
    return out


def oracle_dev(dim, f):
    w = weights(dim)
    return f - w[:, None, None, None]


def compare_fields(g, r, dim, name=""):
    """Return (max |rho_g - rho_o|, max|U_g - U_o| / max|U_o|, max |q_g - q_o|)."""
    drho = float(np.max(np.abs(g["rho"] - r["rho"])))
    Uo = r["U"][:dim]
    du = float(np.max(np.abs(g["U"] - Uo)) / max(np.max(np.abs(Uo)), 1e-300))
    dq = float(np.max(np.abs(g["q"] - r["q"]))) if "q" in g else 0.0
    print(f"[parity {name}] max|drho|={drho:.3e} rel|dU|={du:.3e} max|dq|={dq:.3e} "
          f"max|U|={np.max(np.abs(Uo)):.3e}", flush=True)
    return drho, du, dq
