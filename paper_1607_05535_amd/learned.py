"""Learned per-column corrector of a coarse HEVI run toward a fine run.

Orchestration only: every computation (dynamics, restriction, field
extraction, network inputs, forward/backward/Adam, bounded application) is
a libthor kernel behind the C ABI; this module sequences the calls and owns
the device tensors that hold the stored pairs.

A pair is made from a fine snapshot S: the coarse state R(S) (restriction
onto the coarse grid) is advanced one coarse step, giving C; S is advanced
`ratio` fine steps covering the same time and restricted, giving F.  The
network sees C around each column and learns F - C.
"""
import numpy as np
import torch

from . import thor

N_FIELDS = 5
FIELDS = ("T", "u", "v", "w", "p")


def widths_for(n_lev, hidden=256, layers=3):
    return [7 * N_FIELDS * n_lev] + [hidden] * layers + [N_FIELDS * n_lev]


class Pipeline:
    """fine_w / coarse_w: workload recipes on two grid levels with the same
    planet, levels and forcing; coarse_w.dt = ratio * fine_w.dt."""

    def __init__(self, fine_w, coarse_w, ratio=4, device="cuda:0"):
        assert abs(coarse_w.dt - ratio * fine_w.dt) < 1e-9 * coarse_w.dt
        assert fine_w.n_lev == coarse_w.n_lev and fine_w.z_top == coarse_w.z_top
        self.fw, self.cw, self.ratio, self.device = fine_w, coarse_w, ratio, device
        self.fgrid = thor.Grid(fine_w.glevel)
        self.cgrid = thor.Grid(coarse_w.glevel)
        self.restrict = thor.Restriction(self.fgrid, self.cgrid, device)
        self.N, self.L = self.cgrid.n, coarse_w.n_lev
        self.work = thor.State(self.cgrid, *thor.structs_from_workload(coarse_w), device=device)
        self.ref = thor.State(self.cgrid, *thor.structs_from_workload(coarse_w), device=device)

    def _fine(self, seed):
        from copy import copy
        w = copy(self.fw)
        w.seed = seed
        return thor.State(self.fgrid, *thor.structs_from_workload(w), device=self.device)

    def make_pairs(self, seeds, spinup, pairs_per_seed, log=None):
        """Stored coarse and fine fields, device tensors [n, 5, N, L]."""
        n = len(seeds) * pairs_per_seed
        C = torch.empty(n, N_FIELDS, self.N, self.L, dtype=torch.float32, device=self.device)
        F = torch.empty_like(C)
        k = 0
        for s in seeds:
            fine = self._fine(s)
            fine.step(spinup, self.fw.n_acoustic)
            for _ in range(pairs_per_seed):
                self.restrict(fine, self.work)
                self.work.step(1, self.cw.n_acoustic)
                thor.thor_state_fields32(self.work, C[k])
                fine.step(self.ratio, self.fw.n_acoustic)
                self.restrict(fine, self.ref)
                thor.thor_state_fields32(self.ref, F[k])
                k += 1
            torch.cuda.synchronize()
            if log:
                log(f"pairs from seed {s}: {k}/{n}")
            del fine
        return C, F

    def norm(self, C, F):
        """Means and spreads per (field, level) of the inputs and targets."""
        per = N_FIELDS * self.N * self.L
        a = thor.thor_field_stats(C, None, C.shape[0], per, self.N, self.L)
        b = thor.thor_field_stats(C, F, C.shape[0], per, self.N, self.L)
        for m in (a, b):   # a spread of zero (no variation) is replaced by 1
            m[1] = np.where(m[1] > 0, m[1], 1.0)
        return np.concatenate([a.reshape(-1), b.reshape(-1)]).astype(np.float32)

    def train(self, C, F, norm, steps, batch=4096, lr=1e-3, seed=0, log=None, hidden=256):
        net = thor.MLP(widths_for(self.L, hidden), max(batch, self.N), seed=seed, device=self.device)
        corr = thor.Corrector(self.work, net, norm)
        rs = np.random.default_rng(seed)
        x = torch.empty(batch, 7 * N_FIELDS * self.L, dtype=torch.bfloat16, device=self.device)
        t = torch.empty(batch, N_FIELDS * self.L, dtype=torch.float32, device=self.device)
        per = N_FIELDS * self.N * self.L
        losses = []
        for it in range(steps):
            pairs = torch.from_numpy(rs.integers(0, C.shape[0], batch).astype(np.int32)).to(self.device)
            cols = torch.from_numpy(rs.integers(0, self.N, batch).astype(np.int32)).to(self.device)
            corr.batch(C, F, per, pairs, cols, x, t)
            # cosine decay of the learning rate
            lr_t = lr * 0.5 * (1.0 + np.cos(np.pi * it / steps))
            net.train_step(x, t, max(lr_t, lr * 1e-3))
            if it % max(1, steps // 10) == 0 or it == steps - 1:
                loss, _ = net.loss_grad(x, t, want_grad=False)
                losses.append((it, loss))
                if log:
                    log(f"step {it}: loss {loss:.5f}")
        return net, corr, losses

    def evaluate(self, corr, seeds, spinup, pairs_per_seed):
        """RMS error per field of the plain and of the corrected coarse step
        against the restricted fine run, over held-out snapshots."""
        plain = np.zeros(N_FIELDS)
        fixed = np.zeros(N_FIELDS)
        count = 0
        applied = 0
        buf = torch.empty(3, N_FIELDS, self.N, self.L, dtype=torch.float32, device=self.device)
        for s in seeds:
            fine = self._fine(s)
            fine.step(spinup, self.fw.n_acoustic)
            for _ in range(pairs_per_seed):
                self.restrict(fine, self.work)
                self.work.step(1, self.cw.n_acoustic)
                thor.thor_state_fields32(self.work, buf[0])
                applied += corr.apply()
                thor.thor_state_fields32(self.work, buf[1])
                fine.step(self.ratio, self.fw.n_acoustic)
                self.restrict(fine, self.ref)
                thor.thor_state_fields32(self.ref, buf[2])
                h = buf.double().cpu().numpy()
                plain += np.sum((h[0] - h[2]) ** 2, axis=(1, 2))
                fixed += np.sum((h[1] - h[2]) ** 2, axis=(1, 2))
                count += self.N * self.L
            del fine
        out = {}
        for f, name in enumerate(FIELDS):
            a, b = np.sqrt(plain[f] / count), np.sqrt(fixed[f] / count)
            out[name] = {"rms_plain": float(a), "rms_corrected": float(b), "gain": float(a / b) if b > 0 else None}
        out["columns_corrected_fraction"] = applied / (len(seeds) * pairs_per_seed * self.N)
        return out
