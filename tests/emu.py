"""Run a case through the sanitizer-instrumented host build of the library
(tests/cpu_emu) and read the results back in the layout of helpers.collect.
TEST INFRASTRUCTURE ONLY."""
import ctypes
import os
import subprocess
import sys
import tempfile
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, os.path.join(HERE, "cpu_emu"))


def _params_struct(p):
    from paper_2503_20605_amd import params_from
    return params_from(p)


_build_lock = threading.Lock()


def run_cases(jobs):
    """run_case for each dict of keyword arguments in jobs, as concurrent
    processes; returns the results in order."""
    with ThreadPoolExecutor(max_workers=min(len(jobs), os.cpu_count() or 1)) as ex:
        return list(ex.map(lambda kw: run_case(**kw), jobs))


def run_case(params_list, nodes_list=None, tris_list=None, steps=(1,), storage=0,
             graph_steps=None, shape=None, f0dev=None, forces=None, timing=False,
             inactive=(), rest=None, timeout=600, direct_chunks=False, masks=False,
             contact=None):
    import build as emu_build
    from paper_2503_20605_amd._lib import iblb_diag
    with _build_lock:
        exe = emu_build.build(direct=direct_chunks)
    n = len(params_list)
    nodes_list = nodes_list or [None] * n
    tris_list = tris_list or [None] * n
    f0dev = f0dev or [None] * n
    forces = forces or [None] * n
    dim = params_list[0].dim
    Q = 9 if dim == 2 else 19
    with tempfile.TemporaryDirectory() as d:
        P = (type(_params_struct(params_list[0])) * n)(*[_params_struct(p) for p in params_list])
        open(os.path.join(d, "params.bin"), "wb").write(bytes(P))
        cfg = [f"n {n}", f"storage {storage}", "steps " + ",".join(str(s) for s in steps)]
        if graph_steps is not None:
            cfg.append(f"graph_steps {graph_steps}")
        if shape is not None:
            cfg.append(f"shape {shape}")
        if timing:
            cfg.append("timing 1")
        for k in inactive:
            cfg.append(f"inactive_{k} 1")
        if rest is not None:
            cfg.append("rest " + ",".join(str(v) for v in rest))
        if masks:
            cfg.append("mask 1")
        if contact is not None:
            cfg.append(f"contact {contact[0]!r},{contact[1]!r}")
        for k in range(n):
            lam = float(getattr(params_list[k], "lam", 1.0))
            if lam != 1.0:
                cfg.append(f"lambda_{k} {lam!r}")
            mu_s = float(getattr(params_list[k], "shear", 0.0))
            if mu_s != 0.0:
                cfg.append(f"shear_{k} {mu_s!r}")
            beta = float(getattr(params_list[k], "respace", 0.0))
            if beta != 0.0:
                cfg.append(f"respace_{k} {beta!r}")
            q = nodes_list[k]
            if q is not None:
                q = np.asarray(q, dtype=np.float64)
                cfg.append(f"nodes_{k} {q.shape[0]}")
                np.ascontiguousarray(q.T).tofile(os.path.join(d, f"pos_{k}.bin"))
            t = tris_list[k]
            if t is not None:
                t = np.ascontiguousarray(t, dtype=np.int32)
                cfg.append(f"tris_{k} {t.shape[0]}")
                t.tofile(os.path.join(d, f"tris_{k}.bin"))
            if f0dev[k] is not None:
                cfg.append(f"f0dev_{k} 1")
                np.ascontiguousarray(f0dev[k], dtype=np.float64).tofile(
                    os.path.join(d, f"f0dev_{k}.bin"))
            if forces[k] is not None:
                cfg.append(f"force_{k} 1")
                np.ascontiguousarray(np.asarray(forces[k])[:dim], dtype=np.float32).tofile(
                    os.path.join(d, f"force_{k}.bin"))
        open(os.path.join(d, "config.txt"), "w").write("\n".join(cfg) + "\n")
        env = dict(os.environ)
        # no fake stacks for stack-use-after-return: the harness's fibers
        # would get a fresh one (mapped and unmapped) at every launch, which
        # cost 25 times the run itself; no kernel hands out pointers to its
        # locals
        env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1:detect_stack_use_after_return=0"
        env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
        r = subprocess.run([exe, d], capture_output=True, text=True, timeout=timeout, env=env)
        if r.returncode != 0:
            raise RuntimeError(f"emulated run failed (rc={r.returncode}):\n{r.stderr[-6000:]}")
        status = open(os.path.join(d, "status.txt")).read().split("\n", 1)
        rest_steps = (np.fromfile(os.path.join(d, "rest_steps.bin"), dtype=np.int64)
                      if rest is not None else None)
        outs = []
        for k in range(n):
            p = params_list[k]
            nz = p.nz if dim == 3 else 1
            sh = (nz, p.ny, p.nx)

            def ld(name, dt, shape):
                return np.fromfile(os.path.join(d, f"out_{k}_{name}.bin"), dtype=dt).reshape(shape)

            o = dict(rho=ld("rho", np.float32, sh).astype(np.float64),
                     U=ld("U", np.float32, (dim,) + sh).astype(np.float64),
                     F=ld("F", np.float32, (dim,) + sh).astype(np.float64),
                     fdev=ld("fdev", np.float64, (Q,) + sh))
            if masks and nodes_list[k] is not None:
                for tag in ("inside0", "inside1"):
                    fn = os.path.join(d, f"{tag}_{k}.bin")
                    if os.path.exists(fn):
                        o[tag] = np.fromfile(fn, dtype=np.uint8).reshape(sh)
            if contact is not None and nodes_list[k] is not None:
                o["contact"] = np.fromfile(os.path.join(d, f"contact_{k}.bin"), dtype=np.float64)
            if nodes_list[k] is not None:
                N = np.asarray(nodes_list[k]).shape[0]
                o["q"] = ld("q", np.float64, (dim, N)).T.copy()
                o["qdot"] = ld("qdot", np.float32, (dim, N)).T.astype(np.float64)
                o["phi"] = ld("phi", np.float32, (dim, N)).T.astype(np.float64)
            dg = iblb_diag.from_buffer_copy(open(os.path.join(d, f"out_{k}_diag.bin"), "rb").read())
            o["diag"] = dg.to_dict(dim)
            o["status"] = int(status[0])
            o["message"] = status[1].strip() if len(status) > 1 else ""
            if rest_steps is not None:
                o["rest_steps"] = int(rest_steps[k])
            outs.append(o)
        return outs


def run_mlp(widths, params, x, t, lr=1e-3, timeout=600):
    """One forward, one gradient evaluation and one Adam step of the network
    kernels in the sanitizer build.  Returns (y, grads, loss, params_after)."""
    import build as emu_build
    exe = emu_build.build()
    with tempfile.TemporaryDirectory() as d:
        B = x.shape[0]
        open(os.path.join(d, "config.txt"), "w").write(
            f"mlp 1\nwidths {','.join(str(w) for w in widths)}\nbatch {B}\nlr {lr}\n")
        np.ascontiguousarray(params, dtype=np.float32).tofile(os.path.join(d, "params.bin"))
        np.ascontiguousarray(x, dtype=np.float32).tofile(os.path.join(d, "x.bin"))
        np.ascontiguousarray(t, dtype=np.float32).tofile(os.path.join(d, "t.bin"))
        env = dict(os.environ)
        env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:detect_stack_use_after_return=0"
        env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
        r = subprocess.run([exe, d], capture_output=True, text=True, timeout=timeout, env=env)
        if r.returncode != 0:
            raise RuntimeError(f"emulated network run failed (rc={r.returncode}):\n{r.stderr[-6000:]}")
        y = np.fromfile(os.path.join(d, "y.bin"), dtype=np.float32).reshape(B, widths[-1])
        g = np.fromfile(os.path.join(d, "grads.bin"), dtype=np.float32)
        pa = np.fromfile(os.path.join(d, "params_after.bin"), dtype=np.float32)
        loss = float(open(os.path.join(d, "loss.txt")).read())
        return y, g, loss, pa
