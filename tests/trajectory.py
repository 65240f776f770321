"""Trajectory parity of a single-precision GPU run against the FP64 oracle by replay.

The GPU run is stepped one step at a time (flood_step_n).  Before each step
the GPU exports the wet/dry decision every link of each member is about to
take (flood_get_wet_mask), and after it the step length and end time it used
(flood_get_step_log).  For every member and step:

1. the GPU's decisions equal, bit for bit, the oracle's decisions taken in
   the kernel's precision from the same state (single precision for an FP32
   handle, double in the difference form for an FP64 handle): the kernel
   decides as the wet/dry rule of Eq. 3 says;
2. the FP64 oracle takes the same step (same length, same end time) with the
   same decisions; with the branches of the wet/dry rule aligned the two runs
   differ by rounding only, and every cell and every link is held to the
   tolerances (depth 1e-4 m, discharge 1e-4 of the largest |q|) at every
   checkpoint;
3. the FP64 oracle's own decisions from its replayed state are compared with
   the GPU's: every link where they differ is a flip of the wet/dry rule that
   rounding decides, and is counted with the distance of its FP64 flow depth
   from h_dry;
4. at every checkpoint the step is also re-run in the FP64 oracle from the
   GPU's own state before it (with its decisions): the GPU's result must match
   that one step within the one-step bars (1e-6 m + 4 ulp of the depth, 1e-5 of
   the largest |q|), which holds the kernel's arithmetic of Eqs. 1-3 at every
   checkpoint; a link beyond the trajectory bar is then counted, and the part of
   its distance that the oracle's own step accounts for (the oracle's response
   to the difference between the two input states) is reported;
5. optionally an FP64 run that replays only the step lengths (every link
   deciding itself) is carried along; its distance from the GPU run is
   reported, not held: it is what the flips of 3. do to a trajectory.
"""
import numpy as np

H_TOL = 1e-4     # m
Q_TOL = 1e-4     # of the largest |q| of the reference


def state_error(e, fl, i, ref, catchment=0):
    """(max |dh| m, max |dq| / max|q_ref|, links beyond Q_TOL, cells beyond H_TOL)."""
    gh = e.field(i, fl.FIELD_H, catchment)
    gqx = e.field(i, fl.FIELD_QX, catchment)
    gqy = e.field(i, fl.FIELD_QY, catchment)
    qs = max(np.abs(ref.qx).max(), np.abs(ref.qy).max(), 1e-300)
    dqx = np.abs(gqx - ref.qx)
    dqy = np.abs(gqy - ref.qy)
    dh = np.abs(gh - ref.h)
    n_q = int(np.count_nonzero(dqx > Q_TOL * qs) + np.count_nonzero(dqy > Q_TOL * qs))
    return dh.max(), max(dqx.max(), dqy.max()) / qs, n_q, int(np.count_nonzero(dh > H_TOL))


EXPLAINED = 0.9  # share of an exceeding link's distance the oracle's own step must reproduce


def replay(fl, orc, e, model, refs, t_end, catchment=0, free=None, check_every=25, cap=8192,
           h_tol=H_TOL, q_tol=Q_TOL, mask_mode=1, one_h=1e-6, one_q=1e-5, log=print):
    """Step e to t_end one step at a time, replaying every step of the members in
    refs ({member index: orc.Member at the GPU member's current state}) in the
    oracle as described above.  free: optional {member: orc.Member} replaying the
    step lengths only.  Returns a dict of counts and worst errors."""
    N = e.n_members(catchment)
    members = sorted(refs)
    hdry = model.h_dry
    e.log_steps(cap)
    done = np.zeros(N, dtype=np.int64)
    out = dict(steps=0, mask_links=0, flips=0, flip_gap=0.0, worst_h=0.0, worst_q=0.0, checks=0)

    out.update(q_exceed=0, one_step_h=0.0, one_step_q=0.0, explained=1.0)

    def check(i, one=None):
        """Trajectory bars on member i; one: the oracle's step from the GPU's state."""
        gh = e.field(i, fl.FIELD_H, catchment)
        gqx = e.field(i, fl.FIELD_QX, catchment)
        gqy = e.field(i, fl.FIELD_QY, catchment)
        ref = refs[i]
        qs = max(np.abs(ref.qx).max(), np.abs(ref.qy).max(), 1e-300)
        dh = np.abs(gh - ref.h).max()
        dx_, dy_ = np.abs(gqx - ref.qx), np.abs(gqy - ref.qy)
        dq = max(dx_.max(), dy_.max()) / qs
        out["worst_h"] = max(out["worst_h"], dh)
        out["worst_q"] = max(out["worst_q"], dq)
        out["checks"] += 1
        assert dh <= h_tol, ("member", i, "step", int(done[i]), "dh", dh)
        bx, by = dx_ > q_tol * qs, dy_ > q_tol * qs
        nb = int(bx.sum() + by.sum())
        if one is not None:
            # the kernel's arithmetic from its own state, on every cell and link
            oh = np.abs(gh - one.h)
            tol_h = one_h + 4.0 * np.spacing(np.abs(one.h).astype(np.float32)).astype(np.float64)
            qo = max(np.abs(one.qx).max(), np.abs(one.qy).max(), 1e-300)
            oq = max(np.abs(gqx - one.qx).max(), np.abs(gqy - one.qy).max()) / qo
            out["one_step_h"] = max(out["one_step_h"], oh.max())
            out["one_step_q"] = max(out["one_step_q"], oq)
            assert np.all(oh <= tol_h) and oq <= one_q, ("one step from the GPU state", i, int(done[i]), oh.max(), oq)
            if nb:
                # share of each exceeding link's distance that the oracle's own step
                # from the GPU's input state reproduces: the link moved because its
                # input state moved (by less than the depth bar), not by the kernel's
                # arithmetic, which the one-step bars above hold
                sx = np.abs(one.qx - ref.qx)[bx] / dx_[bx]
                sy = np.abs(one.qy - ref.qy)[by] / dy_[by]
                share = np.concatenate([sx, sy]).min()
                out["explained"] = min(out["explained"], share)
                assert share >= EXPLAINED, ("member", i, "step", int(done[i]), "exceeding link not reproduced", share)
        else:
            assert nb == 0, ("member", i, "step", int(done[i]), "dq", dq, nb)
        out["q_exceed"] += nb

    # small grids re-run every step from the GPU state, so the last step of a member
    # (its end state is checked too) has its one-step re-run
    every_step = model.ny * model.nx <= 200000
    last_one = {}
    while True:
        chk = (out["steps"] + 1) % check_every == 0
        masks = {i: e.wet_mask(i, catchment) for i in members}
        hs = {i: e.field(i, fl.FIELD_H, catchment) for i in members}
        pre = {}
        if chk or every_step:
            for i in members:
                pre[i] = (hs[i], e.field(i, fl.FIELD_QX, catchment), e.field(i, fl.FIELD_QY, catchment))
        e.step_n(t_end, 1)
        dts, tes, cnt = e.step_log(catchment)
        moved = [i for i in members if cnt[i] > done[i]]
        if not moved:
            break
        for i in moved:
            k = int(cnt[i]) - 1
            assert k < cap and cnt[i] == done[i] + 1
            wx, wy = masks[i]
            # 1. the kernel's decisions from its float state, bit for bit
            ox, oy = orc.wet_masks(model, hs[i], refs[i].t, mode=mask_mode)
            assert np.array_equal(ox, wx) and np.array_equal(oy, wy), (
                "member", i, "step", k, "mask mismatches", int((ox != wx).sum() + (oy != wy).sum()))
            out["mask_links"] += wx.size + wy.size
            # 3. the FP64 oracle's own decisions on its replayed state
            rx, ry = orc.wet_masks(model, refs[i].h, refs[i].t)
            fx, fy = rx != wx, ry != wy
            nf = int(fx.sum() + fy.sum())
            if nf:
                hx, hy = orc.link_depths(model, refs[i].h)
                gap = max(np.abs(hx[fx] - hdry).max(initial=0.0), np.abs(hy[fy] - hdry).max(initial=0.0))
                out["flips"] += nf
                out["flip_gap"] = max(out["flip_gap"], gap)
            # 2. the same step in FP64 with the same decisions
            t_pre = refs[i].t
            orc.step_forced(model, refs[i], dts[i, k], tes[i, k], wx, wy)
            last_one.pop(i, None)      # a re-run from an earlier step does not describe this one
            if i in pre:
                one = orc.Member(pre[i][0].copy(), pre[i][1].copy(), pre[i][2].copy(), t=t_pre,
                                 s=refs[i].s, mu=refs[i].mu, class_n=refs[i].class_n, drain_rate=refs[i].drain_rate)
                orc.step_forced(model, one, dts[i, k], tes[i, k], wx, wy)
                pre[i] = one
                last_one[i] = one
            if free is not None and i in free:
                orc.step(model, free[i], dts[i, k])
                free[i].t = tes[i, k]
        done = cnt.copy()
        out["steps"] += 1
        if chk:
            for i in moved:
                check(i, pre[i])
    for i in members:
        assert refs[i].t == t_end
        check(i, last_one.get(i))
    if free is not None:
        out["free"] = {i: state_error(e, fl, i, free[i], catchment) for i in sorted(free)}
    log("replay to t=%g: %d steps, %d link decisions bit-exact, worst |dh| %.3g m, worst |dq| %.3g of max|q|, "
        "%d FP64 decisions differ (flow depth within %.3g m of h_dry); one step from the GPU state: |dh| %.3g m, "
        "|dq| %.3g of max|q|; %d link checks beyond the discharge bar, each at least %.0f %% reproduced by the "
        "oracle's own step from the GPU state"
        % (t_end, out["steps"], out["mask_links"], out["worst_h"], out["worst_q"], out["flips"], out["flip_gap"],
           out["one_step_h"], out["one_step_q"], out["q_exceed"], 100.0 * out["explained"]))
    if free is not None:
        for i, v in out["free"].items():
            log("  member %d, step lengths only: |dh| %.3g m, |dq| %.3g of max|q|, %d links and %d cells beyond "
                "the bars" % (i, v[0], v[1], v[2], v[3]))
    return out
