"""Helpers shared by the GPU parity tests: run a workload through the HIP
library and through the CPU oracle, and compare fields."""
import numpy as np

P_REF = 1.0 / 3.0


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return float(np.linalg.norm(a))
    return float(np.linalg.norm(a - b) / nb)


def oracle_sim(oracle, p, fl):
    return oracle.OracleSim(oracle.make_params(**p), fl["phi"], fl["c"], fl.get("ux"),
                            fl.get("uy"), fl.get("P"))


def gpu_ctx(p_list, fls, precision="fp64", rows=None, graph=True):
    from paper_2504_09024_amd import cmlb
    if isinstance(p_list, dict):
        p_list, fls = [p_list], [fls]
    ctx = cmlb.Context(p_list, precision)
    if isinstance(rows, tuple):
        ctx.set_tile_shape(*rows)
    elif rows:
        ctx.set_tile_rows(rows)
    ctx.set_use_graph(graph)
    for i, fl in enumerate(fls):
        ctx.init_fields(i, fl["phi"], fl["c"], fl.get("ux"), fl.get("uy"), fl.get("P"))
    return ctx


def field_errors(g, o, coupled, moving):
    """Relative L2 per field: phi, c, the velocity u = (ux, uy) as one vector
    field (only where the oracle's u is not identically zero) and, for the
    coupled flow, the pressure P.  ``dP`` (the error of P - P_ref relative to
    the oracle's P - P_ref) is reported as information."""
    err = {"phi": rel_l2(g["phi"], o["phi"]), "c": rel_l2(g["c"], o["c"])}
    if moving:
        gu = np.stack([g["ux"], g["uy"]])
        ou = np.stack([o["ux"], o["uy"]])
        err["u"] = rel_l2(gu, ou)
    if coupled:
        err["P"] = rel_l2(g["P"], o["P"])
        err["dP"] = rel_l2(g["P"] - P_REF, o["P"] - P_REF)
    return err
