"""Forward-Euler steps of the nodal DG discretisation of the transport
equation f_t + xi_x f_x = 0 (Section 5.3) with the state at every spatial
node a third-order Tucker tensor over (xi_x, xi_y, xi_z), and every node's
update sum recompressed on the GPU.

The caller describes the discretisation: `terms[a]` lists the update of
node a as (coefficient, source node, first-mode velocity factor or None),
and `scales` maps each velocity-factor name to a device vector over the
xi_x grid (xi+ = max(xi_x, 0), xi- = min(xi_x, 0) for upwind fluxes).  A
term is the source node's Tucker tensor with its first factor's rows
multiplied by that vector (diag(scale) U_1), which is a Tucker tensor of
the same ranks; every node's scaled first factor comes from one scaling of
all first factors side by side, and is shared by every sum that uses it.  The sums of a step are independent, so each stage of the
sketched sum (Stage 1 sizes, Stages 2-3, Stage 4) runs as one batched
launch sequence over all nodes.
"""
import torch

from . import fortran, round_deterministic, sketch_sum_batched


def euler_sums(states, terms, scales):
    """The per-node update sums of one step as dicts of cores, factors and
    coefficients (the input of sketch_sum_batched).  `states[a]` is the
    (core, [U_1, U_2, U_3]) of node a, float64 on the device."""
    # every node's first factor side by side (one column-major matrix), then
    # one scaling per velocity factor; each node's scaled factor is a view
    u1s = [fortran(us[0]) for _, us in states]
    cols = [0]
    for u in u1s:
        cols.append(cols[-1] + u.shape[1])
    stacked = torch.cat([u.t() for u in u1s], dim=0).t()
    scaled_all = {kind: stacked * v.unsqueeze(1) for kind, v in scales.items()}
    views = {}
    sums = []
    for tl in terms:
        cores, facs, coeffs = [], [], []
        for c, src, kind in tl:
            g, us = states[src]
            if kind is None:
                u1 = us[0]
            else:
                key = (src, kind)
                if key not in views:
                    views[key] = scaled_all[kind][:, cols[src]:cols[src + 1]]
                u1 = views[key]
            cores.append(g)
            facs.append([u1] + list(us[1:]))
            coeffs.append(float(c))
        sums.append({"cores": cores, "factors": facs, "coeffs": coeffs})
    return sums


def euler_step(states, terms, scales, eps, p, kind="krp", seed=0, timings=None):
    """One forward-Euler step with the sketched sum (Algorithm 5 for kind
    "krp", 4 for "kron") at tolerance eps and oversampling p.  Returns the
    new states, the ranks and the sketch sizes of every node.  `timings`: as
    for sketch_sum_batched, plus "sums" (forming the node sums)."""
    t0 = None
    if timings is not None:
        import time
        torch.cuda.synchronize()
        t0 = time.perf_counter()
    sums = euler_sums(states, terms, scales)
    if timings is not None:
        torch.cuda.synchronize()
        timings["sums"] = timings.get("sums", 0.0) + 1e3 * (time.perf_counter() - t0)
    out = sketch_sum_batched(sums, kind, eps, p, seed, timings=timings)
    return [(g, us) for g, us, _, _ in out], [r for _, _, r, _ in out], [s for _, _, _, s in out]


def euler_step_deterministic(states, terms, scales, tau):
    """The same step with the paper's deterministic baseline per node
    (TuckerAxby over all terms, then TuckerRounding with tolerance tau)."""
    new, ranks = [], []
    for x in euler_sums(states, terms, scales):
        g, us, r = round_deterministic(x["cores"], x["factors"], tau, coeffs=x["coeffs"])
        new.append((g, us))
        ranks.append(r)
    return new, ranks


def to_device(states, device):
    """Host (numpy) states of synth-style dicts as float64 device tensors."""
    out = []
    for s in states:
        g = fortran(torch.from_numpy(s["core"]).to(device))
        us = [fortran(torch.from_numpy(u).to(device)) for u in s["factors"]]
        out.append((g, us))
    return out
