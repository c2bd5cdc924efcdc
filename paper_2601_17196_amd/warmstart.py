"""Learned warm start for ASPOT: a small permutation-invariant network that
predicts the duals (u, v) of a POT instance from its two point clouds and
masses (not in the paper: a systems pattern on top of the solver).

Network (one set of weights for both sides; the side of a point shows only
through which set's context it sees):
  features  p = ((x - mu) sqrt(cost_scale), log(n r_i) clipped to [-30, 30], 0)
            mu = mean of all n + m points, so |p_x - p_y|^2 = C_ij
  encoder   h = relu(W2 relu(W1 p + b1) + b2)                  4 -> 128 -> 128
  pooling   ctx_side = mean of h over the side's points
  head      z = relu(W3a h_i + W3b ctx_other + b3)              (128 + 128) -> 128
            gamma u_i = w4 . z + b4                              128 -> 1
The prediction is in cost units; u = prediction / gamma.  w comes from the
exact w-block step of the solver, and the solver keeps the warm start only if
phi(z0) < phi(0).

Inference runs in HIP kernels (pot_warm_predict, BF16 weights and MFMA,
FP32 accumulation).  This module holds the PyTorch definition used to train
the weights on duals the solver itself produced, the exact reference of the
inference arithmetic (used by the tests), and the weight-blob packer.
"""
from __future__ import annotations

import argparse
import os
import time

import numpy as np

HID = 128
NFEAT = 4
HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "warm_c5.npz")

# device blob layout (must match include/pot.h): FP32 biases, then BF16 matrices
F_B1, F_B2, F_B3, F_W4, F_B4 = 0, HID, 2 * HID, 3 * HID, 4 * HID
BF16_OFFSET = 2304                       # bytes
H_W1, H_W2, H_W3A, H_W3B = 0, HID * NFEAT, HID * NFEAT + HID * HID, HID * NFEAT + 2 * HID * HID
BLOB_BYTES = BF16_OFFSET + 2 * (HID * NFEAT + 3 * HID * HID)


def features_np(pts, other, mass, cost_scale):
    """Features of one side (FP64 numpy): pts (n, 2), other (m, 2), mass (n)."""
    allp = np.concatenate([pts, other], 0).astype(np.float64)
    mu = allp.mean(0)
    sc = np.sqrt(cost_scale)
    n = pts.shape[0]
    f = np.zeros((n, NFEAT))
    f[:, :2] = (pts.astype(np.float64) - mu) * sc
    with np.errstate(divide="ignore"):
        f[:, 2] = np.clip(np.log(n * np.asarray(mass, dtype=np.float64)), -30.0, 30.0)
    return f


def make_model():
    import torch.nn as nn

    class WarmNet(nn.Module):
        def __init__(self):
            super().__init__()
            self.enc1 = nn.Linear(NFEAT, HID)
            self.enc2 = nn.Linear(HID, HID)
            self.head_a = nn.Linear(HID, HID)
            self.head_b = nn.Linear(HID, HID, bias=False)
            self.out = nn.Linear(HID, 1)

        def encode(self, f):
            import torch
            return torch.relu(self.enc2(torch.relu(self.enc1(f))))

        def forward(self, fs, ft, ms=None, mt=None):
            """fs (B, n, 4), ft (B, m, 4); optional masks (B, n) / (B, m) of
            valid points.  Returns predictions in cost units (B, n), (B, m)."""
            import torch
            hs, ht = self.encode(fs), self.encode(ft)
            if ms is None:
                cs, ct = hs.mean(1), ht.mean(1)
            else:
                cs = (hs * ms[..., None]).sum(1) / ms.sum(1, keepdim=True)
                ct = (ht * mt[..., None]).sum(1) / mt.sum(1, keepdim=True)
            zs = torch.relu(self.head_a(hs) + self.head_b(ct)[:, None, :])
            zt = torch.relu(self.head_a(ht) + self.head_b(cs)[:, None, :])
            return self.out(zs)[..., 0], self.out(zt)[..., 0]

    return WarmNet()


def state_to_arrays(model):
    sd = {k: v.detach().cpu().double().numpy() for k, v in model.state_dict().items()}
    return {"W1": sd["enc1.weight"], "b1": sd["enc1.bias"], "W2": sd["enc2.weight"], "b2": sd["enc2.bias"],
            "W3a": sd["head_a.weight"], "W3b": sd["head_b.weight"], "b3": sd["head_a.bias"],
            "w4": sd["out.weight"][0], "b4": sd["out.bias"]}


def load_arrays(path=WEIGHTS):
    with np.load(path, allow_pickle=False) as z:
        return {k: np.asarray(z[k], dtype=np.float64) for k in z.files}


def bf16_round(a):
    """FP32 values rounded to BF16 (round to nearest even), as FP32."""
    from . import instances as I
    return I.bf16_bits_to_f64(I.to_bf16_bits(np.asarray(a, dtype=np.float32))).astype(np.float32)


def pack_blob(arr) -> np.ndarray:
    """The device weight blob (uint8) in the layout of include/pot.h."""
    from . import instances as I
    fp = np.zeros(BF16_OFFSET // 4, dtype=np.float32)
    fp[F_B1:F_B1 + HID] = arr["b1"]
    fp[F_B2:F_B2 + HID] = arr["b2"]
    fp[F_B3:F_B3 + HID] = arr["b3"]
    fp[F_W4:F_W4 + HID] = arr["w4"]
    fp[F_B4] = float(np.asarray(arr["b4"]).reshape(-1)[0])
    bf = np.concatenate([I.to_bf16_bits(np.asarray(arr[k], dtype=np.float32)).reshape(-1)
                         for k in ("W1", "W2", "W3a", "W3b")])
    blob = np.concatenate([fp.view(np.uint8), bf.view(np.uint8)])
    assert blob.nbytes == BLOB_BYTES
    return blob


def reference_predict(arr, fs, ft):
    """FP32 reference of the inference kernels on one instance: BF16 weights,
    activations rounded to BF16 where the kernels feed an MFMA, FP32
    accumulation.  fs (n, 4), ft (m, 4) features; returns cost-unit
    predictions (n,), (m,)."""
    W1, W2, W3a, W3b = (bf16_round(arr[k]) for k in ("W1", "W2", "W3a", "W3b"))
    b1, b2, b3, w4 = (np.asarray(arr[k], dtype=np.float32) for k in ("b1", "b2", "b3", "w4"))
    b4 = np.float32(np.asarray(arr["b4"]).reshape(-1)[0])

    def enc(f):
        h1 = np.maximum(f.astype(np.float32) @ W1.T + b1, 0.0)
        h2 = np.maximum(bf16_round(h1) @ W2.T + b2, 0.0)
        return h2

    hs, ht = enc(fs), enc(ft)
    cs, ct = hs.mean(0), ht.mean(0)

    def head(h, ctx_other):
        hb = W3b @ ctx_other + b3
        z = np.maximum(bf16_round(h) @ W3a.T + hb, 0.0)
        return z @ w4 + b4

    return head(hs, ct), head(ht, cs)


# ---------------------------------------------------------------------------
# training on duals produced by the batched solver (run on a GPU)
# ---------------------------------------------------------------------------
def solver_dataset(ks, eps=1e-2, chunk=1024, log=print):
    """Features and cost-unit targets (gamma u, gamma v) of the instances ks of
    the n = m = 256 mixture family, solved by pot_solve_batched (cold)."""
    import torch

    from . import instances as I
    from . import pot
    dev = torch.device("cuda:0")
    FS, FT, TS, TT = [], [], [], []
    for a in range(0, len(ks), chunk):
        insts = [I.c5(k) for k in ks[a:a + chunk]]
        probs = []
        for inst in insts:
            d = pot.to_device_instance(inst, dev, kind="f32", pad_ldc=True)
            probs.append(dict(r=d["r"], c=d["c"], s=d["s"], C=d["C"], kind=d["kind"], ldc=d["ldc"], cmax=1.0))
        st, res, outs = pot.solve_batched(probs, eps, want_uv=True)
        torch.cuda.synchronize()
        for inst, r, (f, g, u, v) in zip(insts, res, outs):
            if r["status"] != 0:
                continue
            FS.append(features_np(inst.x, inst.y, inst.r, inst.cost_scale))
            FT.append(features_np(inst.y, inst.x, inst.c, inst.cost_scale))
            TS.append(r["gamma"] * u.cpu().numpy())
            TT.append(r["gamma"] * v.cpu().numpy())
        log(f"  solved instances {ks[a]}..{ks[min(a + chunk, len(ks)) - 1]} (status {st})")
    return np.stack(FS), np.stack(FT), np.stack(TS), np.stack(TT)


def train(n_train=20000, n_val=1024, epochs=40, batch=64, lr=2e-3, seed=0, out=WEIGHTS, log=print):
    import torch
    torch.manual_seed(seed)
    t0 = time.time()
    log(f"generating {n_train} training and {n_val} validation instances with the solver")
    tr = solver_dataset(list(range(n_train)), log=log)
    va = solver_dataset(list(range(20000, 20000 + n_val)), log=log)
    log(f"data ready in {time.time() - t0:.0f} s: {tr[0].shape[0]} train, {va[0].shape[0]} val")
    dev = torch.device("cuda:0")
    T = [torch.from_numpy(a).float().to(dev) for a in tr]
    V = [torch.from_numpy(a).float().to(dev) for a in va]
    model = make_model().to(dev)
    opt = torch.optim.Adam(model.parameters(), lr=lr)
    steps = epochs * ((T[0].shape[0] + batch - 1) // batch)
    sched = torch.optim.lr_scheduler.OneCycleLR(opt, max_lr=lr, total_steps=steps)
    g = torch.Generator(device="cpu").manual_seed(seed)

    def loss_on(D, idx):
        ps, pt = model(D[0][idx], D[1][idx])
        return ((ps - D[2][idx]) ** 2).mean() + ((pt - D[3][idx]) ** 2).mean()

    for ep in range(epochs):
        perm = torch.randperm(T[0].shape[0], generator=g)
        model.train()
        tot = 0.0
        for a in range(0, len(perm), batch):
            idx = perm[a:a + batch].to(dev)
            loss = loss_on(T, idx)
            opt.zero_grad()
            loss.backward()
            opt.step()
            sched.step()
            tot += float(loss) * len(idx)
        model.eval()
        with torch.no_grad():
            vl = float(loss_on(V, torch.arange(V[0].shape[0], device=dev)))
        log(f"epoch {ep:3d}: train mse {tot / len(perm):.3e}  val mse {vl:.3e}  ({time.time() - t0:.0f} s)")
    arr = state_to_arrays(model)
    np.savez(out, **arr)
    log(f"weights written to {out}")
    return arr


def main():
    ap = argparse.ArgumentParser(description="train the warm-start network on solver-generated duals")
    ap.add_argument("--n-train", type=int, default=20000)
    ap.add_argument("--n-val", type=int, default=1024)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--out", default=WEIGHTS)
    a = ap.parse_args()
    train(a.n_train, a.n_val, a.epochs, out=a.out, log=lambda *x: print(*x, flush=True))


if __name__ == "__main__":
    main()
