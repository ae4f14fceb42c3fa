"""Training data and training loop of the learned tau selector.

Samples (matrix, tau, error) are produced by the library itself: each
recipe matrix is drawn on the device, its exact product formed with FP64
leaves at tau = 0, and SpAMM run at the recipe's thresholds; a sample is
(features(A, A, err), log10(tau / ||A||_F^2)) for every product whose
relative error err lies above twice the leaf-precision floor (where the error
still depends on tau) and below 1e-2.  Every arithmetic step runs in the
library's kernels; this module only sequences the calls.
"""
from __future__ import annotations

import numpy as np

import spamm_inputs as si

from . import (TAU_NFEAT, TauModel, build, generate_decay, multiply, rel_err, tau_features)

SHAPES = [(TAU_NFEAT, 128), (128, 128), (128, 128), (128, 1)]


def training_set(recipes, prec: str = "f32", log=None):
    """(X [N, 515], y [N]) CUDA tensors and per-sample metadata."""
    import torch
    feats, ys, meta = [], [], []
    for i, r in enumerate(recipes):
        A = generate_decay(si.recipe_table(r), r["seed"], r["lo"], r["hi"], r["symmetric"])
        h = build(A, r["leaf"])
        E = multiply(h, h, 0.0, "f64")
        floor = rel_err(multiply(h, h, 0.0, prec), E)
        sroot = float(h.norms(h.levels)[0, 0])
        C = None
        for lt in r["log_tau_rel"]:
            tau = float(10.0 ** lt) * sroot
            C = multiply(h, h, tau, prec, out=C)
            err = rel_err(C, E)
            if 2.0 * floor < err < 1e-2:
                feats.append(tau_features(h, h, err))
                ys.append(float(lt))
                meta.append((i, r["n"], r["leaf"], r["family"], float(lt), err))
        if log and (i + 1) % 50 == 0:
            log(f"tau data: {i + 1}/{len(recipes)} matrices, {len(ys)} samples")
        del A, h, E, C
    X = torch.stack(feats) if feats else torch.empty((0, TAU_NFEAT), device="cuda")
    y = torch.tensor(ys, dtype=torch.float32, device="cuda")
    return X, y, meta


def train_model(X, y, seed: int = 7, epochs: int = 300, batch: int = 256, lr: float = 1e-3, shuffle_seed: int = 11):
    """Train a fresh network (He-initialised from seed) on rows shuffled once on the host."""
    import torch
    perm = np.random.Generator(np.random.PCG64(shuffle_seed)).permutation(X.shape[0])
    idx = torch.from_numpy(perm).to(X.device)
    model = TauModel(si.mlp_init(SHAPES, seed))
    losses = model.train(X[idx].contiguous(), y[idx].contiguous(), epochs, batch, lr)
    return model, losses
