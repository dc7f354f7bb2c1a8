"""Baking a Neural Irradiance Volume on the GPU (Sec. 4.5).

Each step draws training points (80 % uniform in the volume with a uniform
direction, 20 % on surfaces with the surface normal, Sec. 4.2), estimates
their indirect irradiance with the Monte Carlo estimator (culling points
whose first hits are mostly back faces and points with null irradiance),
and takes one Adam step on the Eq. 3 loss; the learning rate is held, then
decays exponentially (Sec. 4.5).  For a model with a scene variable and a
scene that changes with it (Sec. 6), each point also draws its variable t at
random; its target is estimated in the scene at that t and t is the
network's extra input.  This module only sequences library calls;
every step runs in the library's kernels.
"""
import torch

from .niv import McScene, Trainer, MC_NEE, lr_schedule


def lr_at(step, total, lr0=1e-2, lr1=1e-4):
    """The library's Sec. 4.5 schedule (niv_lr_schedule): lr0 held for the
    first fifth of the steps (the paper's 10k of its 50k iterations), then
    exponential decay reaching lr1 at the last step."""
    return lr_schedule(step, total // 5, total, lr0, lr1)


class Baker:
    def __init__(self, niv, params, prims, lo, hi, prec="fp16", batch=1 << 18, spp=256,
                 bounces=3, surface_frac=0.2, seed=0, motion=None):
        self.niv = niv
        self.scene = McScene(prims)
        if motion is not None:
            self.scene.set_motion(motion)
        self.with_t = niv.cfg["n_extra"] > 0
        self.trainer = Trainer(niv, params, prec, max_batch=batch)
        self.lo, self.hi = [float(v) for v in lo], [float(v) for v in hi]
        self.batch, self.spp, self.bounces = batch, spp, bounces
        self.n_surface = int(round(surface_frac * batch))
        self.seed = seed
        dev = params.device
        self.E = torch.empty((batch, 3), dtype=torch.float32, device=dev)
        self.valid = torch.empty(batch, dtype=torch.uint8, device=dev)

    def draw(self, step):
        """Training points (and scene variables) and their Monte Carlo targets
        for one step."""
        pts = self.scene.sample_points(self.lo, self.hi, self.batch, self.n_surface,
                                       seed=(self.seed << 20) + step, device=self.E.device,
                                       with_t=self.with_t)
        x, n = pts[0], pts[1]
        t = pts[2] if self.with_t else None
        self.scene.targets(x, n, self.spp, self.bounces, seed=(self.seed << 20) + step + (1 << 19),
                           flags=MC_NEE, out=(self.E, self.valid), t=t)
        return x, n, t

    def step(self, step, total):
        x, n, t = self.draw(step)
        return self.trainer.step(x, n, self.E, lr_at(step, total), valid=self.valid, extra=t)

    def run(self, total, log_every=0, log=print):
        loss = None
        for s in range(1, total + 1):
            loss = self.step(s, total)
            if log_every and s % log_every == 0:
                log(f"step {s}: loss {float(loss.item()):.4e} lr {lr_at(s, total):.2e}")
        return loss


def held_out_error(niv, model, prec, x, n, E_ref, valid, extra=()):
    """Relative L2 error of the model against reference irradiance on the
    valid held-out points, and the relative MSE of the paper's loss (extra:
    the scene variables of the query)."""
    E, _, _ = niv.query(x, n, model, prec, want_flags=True, extra=extra)
    v = valid.bool()
    d = (E - E_ref)[v].double()
    r = E_ref[v].double()
    rel_l2 = float(torch.linalg.norm(d) / torch.linalg.norm(r))
    relmse = float((d ** 2 / (r ** 2 + 0.01)).mean())
    return rel_l2, relmse
