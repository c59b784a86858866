"""Learned cost model pipeline: train the device MLP on simulator records and
measure the makespan gap its estimates cause against true durations, beside
the per-type average table (the paper's "average execution times")."""
from __future__ import annotations

import numpy as np

from . import synth


def train(mlp, x, log_ticks, n_train, epochs=10, batch=1024, lr=1e-3, log=None):
    """Train on rows [0, n_train) in order, `epochs` passes (device tensors)."""
    import torch
    steps = 0
    for ep in range(epochs):
        # one epoch = n_train // batch Adam steps in order, replayed from a
        # captured graph (bit-identical to a train_step per minibatch)
        mlp.train(x[:n_train], log_ticks[:n_train], batch=batch, epochs=1, lr=lr)
        steps += n_train // batch
        if log:
            torch.cuda.synchronize()
            log(f"epoch {ep + 1}/{epochs} done ({steps} steps)")
    torch.cuda.synchronize()
    return steps


def makespan_gaps(m_true, m_plain, m_learned):
    m_true = np.asarray(m_true, np.float64)
    gp = (np.asarray(m_plain) - m_true) / m_true
    gl = (np.asarray(m_learned) - m_true) / m_true
    return {"gap_plain": float(gp.mean()), "gap_learned": float(gl.mean()),
            "paired_gain": float((gp - gl).mean()), "frac_improved": float((gl < gp).mean()),
            "frac_worse": float((gl > gp).mean())}


def evaluate(dag, workers, b_type, true_ticks, est_mlp, table, tune_key=None, keep_schedules=False):
    """Three batch runs on the same DAGs, all advancing with the true ticks:
    est = true ticks, est = table[type], est = the MLP's estimates.  Each run's
    device status is checked (a failed DAG raises instead of entering the
    gaps with makespan -1).  Returns the makespans per run, and with
    `keep_schedules` also each run's host copy of the schedule."""
    import torch
    from . import inspirit
    dev = est_mlp.device
    dur = torch.from_numpy(np.ascontiguousarray(true_ticks, np.int32)).to(dev)
    est_tab = torch.from_numpy(np.ascontiguousarray(table[b_type], np.int32)).to(dev)
    out, scheds = {}, {}
    for name, est in (("true", dur), ("plain", est_tab), ("learned", est_mlp)):
        o = inspirit.schedule_batch(dag, workers, dur, est, tune_key=tune_key)
        inspirit.sync_status(dag)
        ms = o["makespan"].cpu().numpy().copy()
        if (ms < 0).any():
            raise RuntimeError(f"cost-model evaluation: {int((ms < 0).sum())} DAGs failed in the '{name}' run")
        out[name] = ms
        if keep_schedules:
            n = int(dag.task_off[-1])
            scheds[name] = {k: o[k][:n].cpu().numpy() for k in ("worker", "start", "finish")}
            scheds[name]["makespan"] = ms
    return (out, scheds) if keep_schedules else out
