"""The learned cost model as the oracle sees it (test infrastructure): the
FP64 reference network trained from the seeded initial parameters on
simulator records, its integer estimates for a sample of the 4096-DAG batch,
and the per-type table, computed once per test process."""
from __future__ import annotations

import functools

import numpy as np

from oracle import mlp
from paper_2404_03226_amd import synth

RECORDS = 100_000     # training records (90% train, 10% validation)
EPOCHS = 2            # 174 Adam steps of 1024 records
LR = 2e-3
SAMPLE = list(range(0, 4096, 128))  # 32 DAGs of the batch, ~140k tasks


@functools.lru_cache(maxsize=None)
def trained():
    """(records, float64 parameters, Adam steps, per-type table)."""
    rec = synth.cfg5_records(n=RECORDS)
    ntr = rec["n_train"]
    T = np.log(rec["ticks"].astype(np.float64))
    params, steps = mlp.train(synth.mlp_init(), rec["x"][:ntr], T[:ntr], batch=1024, epochs=EPOCHS, lr=LR)
    table = synth.plain_table(rec["types"][:ntr], rec["ticks"][:ntr])
    return rec, params, steps, table


@functools.lru_cache(maxsize=None)
def sample():
    """The sampled DAGs (types read as Cholesky kernels), their features, true
    ticks, and the three estimate tables: truth, the per-type table, and the
    reference network's integer estimates."""
    _, params, _, table = trained()
    ws = synth.cfg3(select=SAMPLE)
    b = synth.concat(ws)
    x = synth.cost_features(5, 7, b.type)
    ticks = synth.cost_truth(5, 7, b.type, x)
    est = {"true": ticks, "plain": np.ascontiguousarray(table[b.type], np.int32),
           "learned": mlp.ticks_from_log(mlp.forward(params, x, bf=True)["Y"])}
    return ws, b, x, ticks, est
