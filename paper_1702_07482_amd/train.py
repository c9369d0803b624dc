"""Training driver: the loss and the two training schedules of Sec. 2.2.2.

The trainable parameters of a T-stage model are the filters k_i^t, the RBF
weights w_ij^t and, for each stage, beta^t with lambda^t = exp(beta^t) (Sec. 3.2:
training works on beta so that lambda stays positive; the chain rule gives
dl/dbeta = lambda dl/dlambda, eq. derv5).  The loss over S training pairs is
    L(Theta) = sum_s 1/2 || u_T^s - u_gt^s ||^2        (eq. learning).
Every forward and gradient comes from libtnrd (tnrd_forward / tnrd_backward
through autograd.TNRDFunction); this module only runs the optimiser.

* train_joint: all stages at once with L-BFGS (strong Wolfe line search).
* train_greedy: stage by stage; stage t is fitted on the loss at u_t with the
  stages before it frozen, which gives the joint training its initialisation.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from .autograd import tnrd_apply


class TrainableModel(torch.nn.Module):
    """filters [T][Nk][k][k], rbf_w [T][Nk][Nrbf], beta [T] as CUDA parameters."""

    def __init__(self, filters, rbf_w, lam, mu0=-310.0, step=10.0, sigma=10.0, L=1,
                 reaction="prox", proj_c=1.0, opts=None, device="cuda"):
        super().__init__()
        t = lambda a: torch.as_tensor(a, dtype=torch.float32, device=device).clone()
        self.filters = torch.nn.Parameter(t(filters))
        self.rbf_w = torch.nn.Parameter(t(rbf_w))
        self.beta = torch.nn.Parameter(torch.log(t(lam)))
        self.meta = dict(mu0=float(mu0), step=float(step), sigma=float(sigma), L=int(L),
                         reaction=reaction, proj_c=float(proj_c), opts=opts)

    @classmethod
    def from_dict(cls, m: dict, L: int = 1, **kw) -> "TrainableModel":
        return cls(m["filters"], m["rbf_w"], m["lam"], m["mu0"], m["step"], m["sigma"], L=L,
                   reaction=m.get("reaction", "prox"), proj_c=m.get("proj_c", 1.0), **kw)

    @property
    def T(self) -> int:
        return int(self.filters.shape[0])

    def lam(self) -> torch.Tensor:
        return torch.exp(self.beta)

    def forward(self, f: torch.Tensor, stages: int | None = None, params=None) -> torch.Tensor:
        """u_t after the first `stages` stages (all by default); `params` may
        replace (filters, rbf_w, beta) for those stages."""
        K, Wt, B = params if params is not None else (self.filters, self.rbf_w, self.beta)
        s = self.T if stages is None else int(stages)
        return tnrd_apply(f, K[:s].contiguous(), Wt[:s].contiguous(), torch.exp(B[:s]).contiguous(),
                          **self.meta)

    def to_dict(self) -> dict:
        m = {"filters": self.filters.detach().cpu().numpy(), "rbf_w": self.rbf_w.detach().cpu().numpy(),
             "lam": self.lam().detach().cpu().numpy()}
        m.update({k: self.meta[k] for k in ("mu0", "step", "sigma", "reaction", "proj_c")})
        m.update({"T": self.T, "Nk": int(self.filters.shape[1]), "ks": int(self.filters.shape[2]),
                  "Nrbf": int(self.rbf_w.shape[2])})
        return m


def loss_fn(u: torch.Tensor, u_gt: torch.Tensor) -> torch.Tensor:
    """1/2 sum over pairs and pixels of (u_T - u_gt)^2."""
    return 0.5 * ((u - u_gt) ** 2).sum()


@dataclass
class TrainLog:
    losses: list = field(default_factory=list)   # loss at every evaluation
    stages: list = field(default_factory=list)   # stage trained at that evaluation (0 = joint)


def train_joint(model: TrainableModel, f: torch.Tensor, u_gt: torch.Tensor, iters: int = 20,
                history: int = 10, log: TrainLog | None = None) -> TrainLog:
    """Joint training of every stage with L-BFGS on the batch f -> u_gt ([S][H][W])."""
    log = log or TrainLog()
    opt = torch.optim.LBFGS(model.parameters(), lr=1.0, max_iter=iters, history_size=history,
                            line_search_fn="strong_wolfe")

    def closure():
        opt.zero_grad()
        loss = loss_fn(model(f), u_gt)
        loss.backward()
        log.losses.append(float(loss.detach()))
        log.stages.append(0)
        return loss

    opt.step(closure)
    return log


def train_greedy(model: TrainableModel, f: torch.Tensor, u_gt: torch.Tensor, iters: int = 10,
                 history: int = 10, log: TrainLog | None = None) -> TrainLog:
    """Stage-by-stage training: stage t (1..T) minimises the loss at u_t over its own
    parameters, the earlier stages frozen at their trained values."""
    log = log or TrainLog()
    for t in range(1, model.T + 1):
        k_t = torch.nn.Parameter(model.filters.detach()[t - 1].clone())
        w_t = torch.nn.Parameter(model.rbf_w.detach()[t - 1].clone())
        b_t = torch.nn.Parameter(model.beta.detach()[t - 1:t].clone())
        opt = torch.optim.LBFGS([k_t, w_t, b_t], lr=1.0, max_iter=iters, history_size=history,
                                line_search_fn="strong_wolfe")

        def params():
            K = torch.cat([model.filters.detach()[:t - 1], k_t[None]])
            Wt = torch.cat([model.rbf_w.detach()[:t - 1], w_t[None]])
            B = torch.cat([model.beta.detach()[:t - 1], b_t])
            return K, Wt, B

        def closure():
            opt.zero_grad()
            loss = loss_fn(model(f, stages=t, params=params()), u_gt)
            loss.backward()
            log.losses.append(float(loss.detach()))
            log.stages.append(t)
            return loss

        opt.step(closure)
        with torch.no_grad():
            model.filters[t - 1].copy_(k_t)
            model.rbf_w[t - 1].copy_(w_t)
            model.beta[t - 1:t].copy_(b_t)
    return log
