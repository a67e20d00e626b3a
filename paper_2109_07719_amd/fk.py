"""Forward kinematics of link points in torch (loss-side helper).

Losses on the end state of a rollout (for example an end-effector target)
are ordinary differentiable torch code; their gradient with respect to q^T
becomes the seed of the adjoint pass (Sec. 3, Eq. diff_u: dPhi/dx^T enters
the adjoint recursion).  This module computes world positions of chosen
points on chosen links for a whole batch, one tree level at a time, with the
package's joint convention (revolute: link -> parent rotation
E^T = E_T^T Rot(a, q), Rot the rotation by +q about a, origin at r_T;
prismatic: E^T = E_T^T, origin at r_T + q E_T^T a; spherical: E^T =
E_T^T R(quat), origin at r_T; free root: R(quat) and p).  Other joint types
are rejected.
"""
from __future__ import annotations

import numpy as np
import torch


def _skew(a):
    z = torch.zeros_like(a[..., 0])
    return torch.stack([torch.stack([z, -a[..., 2], a[..., 1]], -1),
                        torch.stack([a[..., 2], z, -a[..., 0]], -1),
                        torch.stack([-a[..., 1], a[..., 0], z], -1)], -2)


def _quat_R(qt):
    x, y, z, w = qt.unbind(-1)
    return torch.stack([
        torch.stack([w * w + x * x - y * y - z * z, 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), w * w - x * x + y * y - z * z, 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), w * w - x * x - y * y + z * z], -1)], -2)


class LinkPoints(torch.nn.Module):
    """World positions of one point per system: point `pts[s]` (link
    coordinates) on link `links[s]` (local index) of system s."""

    def __init__(self, systems, links, pts, dtype=torch.float32, device="cuda"):
        super().__init__()
        glob_par, dep, qidx, jt, ET, rT, ax, target = [], [], [], [], [], [], [], []
        base, qbase = 0, 0
        for s, sy in enumerate(systems):
            d = sy.depth()
            qo = 0
            for i in range(sy.n):
                if int(sy.jtype[i]) not in (0, 1, 2, 3):
                    raise ValueError(f"LinkPoints: system {s} link {i} has joint type {int(sy.jtype[i])}; "
                                     "only revolute (0), free root (1), prismatic (2) and spherical (3) "
                                     "joints are supported")
                glob_par.append(-1 if sy.parent[i] < 0 else base + int(sy.parent[i]))
                dep.append(int(d[i]))
                qidx.append(qbase + qo)
                jt.append(int(sy.jtype[i]))
                ET.append(np.asarray(sy.E_T[i]))
                rT.append(np.asarray(sy.r_T[i]))
                ax.append(np.asarray(sy.axis[i]))
                qo += 7 if sy.jtype[i] == 1 else 4 if sy.jtype[i] == 3 else 1
            target.append(base + int(links[s]))
            base += sy.n
            qbase += qo
        f = lambda x: torch.tensor(np.asarray(x), dtype=dtype, device=device)
        i64 = lambda x: torch.tensor(np.asarray(x), dtype=torch.long, device=device)
        self.n_links = base
        self.parent = i64(glob_par)
        self.depth = np.asarray(dep)
        self.qidx = i64(qidx)
        self.qidx_np = np.asarray(qidx)
        self.jtype = np.asarray(jt)
        self.ETt = f(np.stack(ET)).transpose(-1, -2).contiguous()
        self.rT = f(np.stack(rT))
        self.K = _skew(f(np.stack(ax)))
        self.ax = f(np.stack(ax))
        self.prism = torch.tensor(np.asarray(jt) == 2, device=device)
        self.target = i64(target)
        self.pts = f(np.asarray(pts))
        self.levels = [torch.tensor(np.nonzero(self.depth == d)[0], dtype=torch.long, device=device)
                       for d in range(int(self.depth.max()) + 1)]
        self.level_free = [np.nonzero(self.jtype[np.nonzero(self.depth == d)[0]] == 1)[0]
                           for d in range(int(self.depth.max()) + 1)]
        self.level_ball = [np.nonzero(self.jtype[np.nonzero(self.depth == d)[0]] == 3)[0]
                           for d in range(int(self.depth.max()) + 1)]

    def forward(self, q):
        n = self.n_links
        Rw = torch.zeros((n, 3, 3), dtype=q.dtype, device=q.device)
        pw = torch.zeros((n, 3), dtype=q.dtype, device=q.device)
        I3 = torch.eye(3, dtype=q.dtype, device=q.device)
        for idx, free, ball in zip(self.levels, self.level_free, self.level_ball):
            m = idx.numel()
            qi = q[self.qidx[idx]]
            K = self.K[idx]
            pr = self.prism[idx]
            s, c = torch.sin(qi)[:, None, None], torch.cos(qi)[:, None, None]
            Rj = torch.where(pr[:, None, None], I3.expand(m, 3, 3), I3 + s * K + (1 - c) * (K @ K))
            if len(ball):
                rows = list(Rj.unbind(0))
                for k in ball:
                    qo = int(self.qidx_np[int(idx[k])])
                    rows[k] = _quat_R(q[qo:qo + 4])
                Rj = torch.stack(rows)
            par = self.parent[idx]
            has_par = par >= 0
            parc = par.clamp(min=0)
            Rp = torch.where(has_par[:, None, None], Rw[parc], I3.expand(m, 3, 3))
            pp = torch.where(has_par[:, None], pw[parc], torch.zeros((m, 3), dtype=q.dtype, device=q.device))
            Rl = Rp @ self.ETt[idx] @ Rj
            # a prismatic link's origin slides by q a (joint frame) from r_T
            slide = torch.where(pr[:, None], qi[:, None] * self.ax[idx], torch.zeros_like(self.ax[idx]))
            r = self.rT[idx] + (self.ETt[idx] @ slide[..., None])[..., 0]
            pl = pp + (Rp @ r[..., None])[..., 0]
            if len(free):
                rows_R, rows_p = list(Rl.unbind(0)), list(pl.unbind(0))
                for k in free:
                    qo = int(self.qidx_np[int(idx[k])])
                    rows_R[k] = _quat_R(q[qo + 3:qo + 7])
                    rows_p[k] = q[qo:qo + 3]
                Rl, pl = torch.stack(rows_R), torch.stack(rows_p)
            Rw = Rw.index_copy(0, idx, Rl)
            pw = pw.index_copy(0, idx, pl)
        t = self.target
        return pw[t] + (Rw[t] @ self.pts[..., None])[..., 0]
