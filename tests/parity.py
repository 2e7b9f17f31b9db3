"""Shared helpers of the GPU parity tests: run the C-ABI library and the
oracle on the same inputs and compare element by element.

Tolerances (FP32 path against the FP64 oracle):
  distance   |d - d_o| <= 1e-4 m
  gradient   max_i |g_i - g_o,i| <= 1e-3
  variance   |v / v_o - 1| <= 2e-3 (the FP32 path sends queries whose
             estimated relative variance error exceeds 1e-3 to FP64; 2e-3
             leaves a factor 2 for the estimate)
  validity, n_local: exact
  sign: equal except at the oracle's sign near-ties (queries whose nearest
        training points on different sides of the surface lie within FP32
        rounding of each other), which are counted
FP64 path: FP64-level agreement plus the final rounding of the FP32 outputs.
"""
import numpy as np
import torch

import oracle as O
import paper_2407_09649_amd as P

TOL_D, TOL_G, TOL_V = 1e-4, 1e-3, 2e-3


def small_params(**kw):
    base = dict(max_points=1 << 20, max_clusters=1 << 16, max_queries=1 << 20,
                global_capacity=1 << 20, max_factor_elems=1 << 23)
    base.update(kw)
    return P.Params.default(**base)


def oracle_params(p: P.Params) -> O.Params:
    return O.Params(kernel=p.kernel, selection=p.selection, knn_q=p.knn_q,
                    combine=p.combine, grad_mode=p.grad_mode, l=p.length_scale,
                    s=p.noise_sigma, voxel=p.voxel_size, cell=p.cluster_size,
                    lam=p.smooth_min_lambda, occ_min=p.occ_min, occ_max=p.occ_max,
                    fuse_voxel=p.fuse_voxel_size, fuse_band=p.fuse_band,
                    fuse_rule=p.fuse_rule, tp_mode=p.test_points, normal_reach=p.normal_reach)


def gpu_query(ctx, q, origin=None):
    dev = ctx.device
    r = ctx.query(torch.from_numpy(np.ascontiguousarray(q, np.float32)).to(dev), origin=origin)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in r.items()}


def _node_alt(g, o, v, s):
    """Closest-node rule: at the oracle's node near-ties (second-closest
    node within 2e-4 m of the closest) an FP32 argmin may pick the other
    node.  Returns g's distance, gradient and variance (and property) with
    those queries replaced by the oracle's answer it matches better, so
    that both valid answers pass and nothing else does."""
    nt = np.asarray(o.get("node_tie", np.zeros(len(v), bool)))[v]
    ref = {k: np.array(o[k][v], copy=True) for k in ("dist", "grad", "var", "prop", "prop_var") if k in o}
    if not nt.any():
        return ref, 0
    alt = {k: np.asarray(o["alt"][k])[v] for k in ref}
    sg = np.where(np.sign(g["dist"][v]) != np.sign(o["dist"][v]), -1.0, 1.0)
    e0 = np.abs(sg * g["dist"][v] - ref["dist"]) + np.abs(sg[:, None] * g["grad"][v] - ref["grad"]).max(1)
    e1 = np.abs(sg * g["dist"][v] - alt["dist"]) + np.abs(sg[:, None] * g["grad"][v] - alt["grad"]).max(1)
    use = nt & (e1 < e0)
    for k in ref:
        ref[k][use] = alt[k][use]
    return ref, int(use.sum())


def compare(g, o, fp64=False, check_aux=True, label="", closest_node=False):
    """Element-wise comparison; returns a dict of maximum errors and the sign
    counts.  The oracle decides the sign from the exact nearest training point
    and flags the queries whose decision an FP32 evaluation can take the other
    way (``sign_tie``); a sign may differ only there, and the magnitude and
    gradient are still compared with the sign aligned.  closest_node: the
    closest-node rule, where a node near-tie admits the oracle's second answer
    (``alt``), counted in ``node_alt``."""
    vg = g["valid"].astype(bool)
    vo = np.asarray(o["valid"]).astype(bool)
    assert (vg == vo).all(), f"{label}: validity differs on {(vg != vo).sum()} queries"
    v = vo
    inval = ~v
    assert np.isinf(g["dist"][inval]).all() and (g["grad"][inval] == 0).all()
    out = dict(n=int(v.sum()), sign_ties=0, sign_flips=0)
    if not v.any():
        return out
    tie = np.asarray(o.get("sign_tie", np.zeros(len(vo), bool)))[v]
    flip = np.sign(g["dist"][v]) != np.sign(o["dist"][v])
    assert not (flip & ~tie).any(), f"{label}: sign differs on {(flip & ~tie).sum()} queries with no near-tie"
    s = np.where(flip, -1.0, 1.0)
    out.update(sign_ties=int(tie.sum()), sign_flips=int(flip.sum()))
    if closest_node and not fp64:
        ref, out["node_alt"] = _node_alt(g, o, v, s)
    else:
        ref = {k: o[k][v] for k in ("dist", "grad", "var", "prop", "prop_var") if k in o}
    out["ref"] = ref
    d_err = np.abs(s * g["dist"][v] - ref["dist"])
    g_err = np.abs(s[:, None] * g["grad"][v] - ref["grad"]).max(1)
    v_rel = np.abs(g["var"][v] / ref["var"] - 1.0)
    out.update(d=float(d_err.max()), g=float(g_err.max()), v=float(v_rel.max()))
    if fp64:
        # FP64 arithmetic, results stored as FP32: one rounding (2^-24
        # relative) on top of FP64-level agreement
        u = 2.0 ** -24
        assert (d_err <= 1e-9 + 2 * u * np.abs(o["dist"][v])).all(), (label, d_err.max())
        gmax = np.abs(o["grad"][v]).max(1)
        assert (g_err <= 1e-8 + 2 * u * gmax).all(), (label, g_err.max())
        assert (v_rel <= 1e-8 + 2 * u).all(), (label, v_rel.max())
    else:
        assert (d_err <= TOL_D).all(), (label, d_err.max())
        assert (g_err <= TOL_G).all(), (label, g_err.max())
        assert (v_rel <= TOL_V).all(), (label, v_rel.max())
    if check_aux:
        assert (g["aux"][v, 2] == o["aux"][v, 2]).all(), f"{label}: n_local differs"
    print(f"{label}: {out['n']} valid, sign near-ties {out['sign_ties']}, sign flips {out['sign_flips']}, "
          f"other closest node {out.get('node_alt', 0)}, "
          f"max errors d {out['d']:.3g} g {out['g']:.3g} v {out['v']:.3g}")
    return out


def signed_dist_err(gdist, o, label=""):
    """|d - d_o| over the oracle's valid queries with the sign aligned where
    the oracle reports a sign near-tie (a sign may differ only there)."""
    v = np.asarray(o["valid"]).astype(bool)
    tie = np.asarray(o.get("sign_tie", np.zeros(len(v), bool)))[v]
    g = np.asarray(gdist)[v]
    flip = np.sign(g) != np.sign(o["dist"][v])
    assert not (flip & ~tie).any(), f"{label}: sign differs on {(flip & ~tie).sum()} queries with no near-tie"
    return np.abs(np.where(flip, -g, g) - o["dist"][v])


def export_equal(ctx, om, alpha_rtol=1e-9):
    e = ctx.export_model()
    eo = om.export()
    assert np.array_equal(e["ckey"], eo["ckey"]), "cluster keys differ"
    assert np.array_equal(e["off"], eo["off"]), "cluster offsets differ"
    assert np.array_equal(e["points"].view(np.uint32), eo["points"].view(np.uint32)), \
        "training points differ"
    assert np.array_equal(e["pd"], eo["pd"])
    scale = np.abs(eo["alpha"]).max() if eo["alpha"].size else 1.0
    assert np.abs(e["alpha"] - eo["alpha"]).max(initial=0.0) <= alpha_rtol * scale
    return e
