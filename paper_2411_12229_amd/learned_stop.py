"""Training of the learned early stop used by ``qg_search_stop``.

The plain search (Algorithm 1) keeps expanding until its beam has no unchecked
entry.  The learned stop ends a query early: after the t-th expansion (t >=
t_min, every t_every) a 16-64-64-1 ReLU MLP reads 16 features of the search
state and the query stops when its output exceeds theta.

Training data come from the device kernel itself: ``Index.search_stop`` with
no model writes, at every evaluation point, the features and the current top-k
ids.  A point is labelled 1 when stopping there keeps the recall the query
reaches by running to the end, so the MLP learns "nothing more will be found".
Parameters are exported as bf16 bit patterns (round to nearest even) in the
layout W1[64][16], b1[64], W2[64][64], b2[64], W3[64], b3.
"""
from __future__ import annotations

import torch

N_PARAMS = 64 * 16 + 64 + 64 * 64 + 64 + 64 + 1


def recall_rows(ids: torch.Tensor, gt: torch.Tensor) -> torch.Tensor:
    """|ids[..., :] ∩ gt| / k for ids [..., k] against gt [nq, k] broadcast over the middle dims."""
    k = gt.shape[-1]
    g = gt.view(gt.shape[0], *([1] * (ids.dim() - 2)), 1, k)
    hit = (ids.unsqueeze(-1) == g).any(-1) & (ids >= 0)
    return hit.sum(-1).float() / k


def collect(idx, queries: torch.Tensor, gt: torch.Tensor, k: int, ef: int, t_min: int, t_every: int,
            trace_max: int = 128):
    """Trace the plain search; return (features [M,16], labels [M]) on the queries' device."""
    ids, _, _, tr = idx.search_stop(queries, k, ef, None, t_min=t_min, t_every=t_every, trace_max=trace_max)
    feat, nn, _, cnt = tr
    final = recall_rows(ids, gt)                       # [nq]
    rec = recall_rows(nn, gt)                           # [nq, T]
    T = feat.shape[1]
    valid = torch.arange(T, device=feat.device)[None, :] < cnt[:, None]
    label = (rec >= final[:, None]).float()
    return feat[valid], label[valid]


def ideal_stop(idx, queries: torch.Tensor, gt: torch.Tensor, k: int, ef: int, t_min: int, t_every: int,
               trace_max: int = 256):
    """The bound any stop rule evaluated at these points can reach: each query stops at the first evaluation
    point whose top-k already has the recall the full search ends with (recall unchanged).  Returns (mean
    expansions with that stop, mean expansions of the full search)."""
    ids, _, st, tr = idx.search_stop(queries, k, ef, None, t_min=t_min, t_every=t_every, trace_max=trace_max,
                                     stats=True)
    _, nn, _, cnt = tr
    final = recall_rows(ids, gt)
    rec = recall_rows(nn, gt)
    T = nn.shape[1]
    pts = torch.arange(T, device=nn.device)
    done = (rec >= final[:, None]) & (pts[None, :] < cnt[:, None])
    first = torch.where(done.any(1), done.float().argmax(1), torch.full_like(cnt, T).long())
    full = st[:, 0].float()
    at = torch.where(first < T, (t_min + first * t_every).float(), full)
    return torch.minimum(at, full).mean().item(), full.mean().item()


class StopMLP(torch.nn.Module):
    def __init__(self):
        super().__init__()
        self.l1 = torch.nn.Linear(16, 64)
        self.l2 = torch.nn.Linear(64, 64)
        self.l3 = torch.nn.Linear(64, 1)

    def forward(self, x):
        return self.l3(torch.relu(self.l2(torch.relu(self.l1(x))))).squeeze(-1)


def train(features: torch.Tensor, labels: torch.Tensor, epochs: int = 8, batch: int = 8192, lr: float = 3e-3,
          seed: int = 0) -> StopMLP:
    torch.manual_seed(seed)
    dev = features.device
    model = StopMLP().to(dev)
    opt = torch.optim.Adam(model.parameters(), lr=lr)
    n = features.shape[0]
    g = torch.Generator(device=dev).manual_seed(seed)
    for _ in range(epochs):
        perm = torch.randperm(n, device=dev, generator=g)
        for s in range(0, n, batch):
            i = perm[s:s + batch]
            loss = torch.nn.functional.binary_cross_entropy_with_logits(model(features[i]), labels[i])
            opt.zero_grad()
            loss.backward()
            opt.step()
    return model


def to_bf16_bits(x: torch.Tensor) -> torch.Tensor:
    """fp32 -> bf16 bit patterns, round to nearest even (int16 view of the bits)."""
    return x.detach().float().contiguous().to(torch.bfloat16).view(torch.int16)


def export(model: StopMLP) -> torch.Tensor:
    """Flat bf16 parameter vector (int16 bits) in the kernel's layout."""
    parts = [model.l1.weight, model.l1.bias, model.l2.weight, model.l2.bias, model.l3.weight.view(-1),
             model.l3.bias]
    w = torch.cat([to_bf16_bits(p).view(-1) for p in parts])
    assert w.numel() == N_PARAMS
    return w.contiguous()


def pick_theta(idx, queries: torch.Tensor, gt: torch.Tensor, mlp_bits: torch.Tensor, k: int, ef: int, t_min: int,
               t_every: int, target: float, grid=None):
    """Largest stopping eagerness (smallest theta) whose recall on these queries reaches target.
    Returns (theta, recall, mean expansions) or None."""
    def at(th):
        ids, _, st, _ = idx.search_stop(queries, k, ef, mlp_bits, theta=th, t_min=t_min, t_every=t_every,
                                        stats=True)
        return th, recall_rows(ids, gt).mean().item(), st[:, 0].float().mean().item()

    best, fail = None, None
    for th in (grid if grid is not None else [6.0 - 0.25 * i for i in range(33)]):
        got = at(th)
        if got[1] < target:
            fail = th
            break
        best = got
    # between the last theta that reaches the target and the first that does not,
    # in steps of 0.05 (the default grid only)
    if grid is None and best is not None and fail is not None:
        th = best[0] - 0.05
        while th > fail + 1e-9:
            got = at(round(th, 2))
            if got[1] < target:
                break
            best = got
            th -= 0.05
    return best
