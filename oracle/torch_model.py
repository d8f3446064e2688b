"""Vectorised FP64 PyTorch (CPU) form of the same lattice Boltzmann step, for
reverse-mode gradients through many steps (the oracle adjoint).

TEST INFRASTRUCTURE ONLY (imported by tests and the benchmark's checks; never
by the GPU library or its binding). It shares no code with the C oracle or
with the HIP path: it is a second, whole-array statement of Sec. 2 of the
paper, in pull form, for flat walls (no solid cells inside the lattice):

  pull with half-way bounce-back (f) / anti-bounce-back at T_w (g), moments
  (Eqs. (4), (5), (17)), pseudopotentials psi_x = rho/rho0 (Eq. (8)) and
  psi_s = rho0 (1 - exp(-rho/rho0)) (Eq. (12)) with two wall ghost rows at
  the wetting densities (Sec. 2.2.1), forces (Eqs. (7), (10), (11), (22)),
  velocity shift (Eq. (6)), u^H = u + F/(2 rho), BGK collision (Eqs. (2),
  (3), (16), (18)).

The state is the post-collision populations f*(t) (three [9, ly, lx]
tensors), so that one call of `step` maps f*(t) to f*(t+1) exactly as the
GPU library's state advances. The loss used for the adjoint is the time
average of the top-wall Nusselt number (Sec. 3.3.2, top-wall flux form).

Parity: pinned by tests against the C oracle's forward and against central
finite differences of its own gradient.
"""
from __future__ import annotations

import math

import torch

CX = (0, 1, 0, -1, 0, 1, -1, -1, 1)
CY = (0, 0, 1, 0, -1, 1, 1, -1, -1)
OPP = (0, 3, 4, 1, 2, 7, 8, 5, 6)
W = (4 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 36, 1 / 36, 1 / 36, 1 / 36)
CS2 = 1.0 / 3.0


def _p_weight(c2: int) -> float:
    """25-point weights of Fig. 1(b) by |c|^2."""
    return {0: 247 / 420, 1: 4 / 63, 2: 4 / 135, 4: 1 / 180, 5: 2 / 945, 8: 1 / 15120}[c2]


def _w_weight(c2: int) -> float:
    return {0: 4 / 9, 1: 1 / 9, 2: 1 / 36}.get(c2, 0.0)


class Model:
    """Constants and geometry of one lattice (flat walls below and above)."""

    def __init__(self, params: dict, lx: int, ly: int):
        self.p = params
        self.lx, self.ly = lx, ly
        self.w = torch.tensor(W, dtype=torch.float64).view(9, 1, 1)
        self.cx = torch.tensor(CX, dtype=torch.float64).view(9, 1, 1)
        self.cy = torch.tensor(CY, dtype=torch.float64).view(9, 1, 1)

    # ---------------------------------------------------------------- pieces
    def equilibrium(self, rho, ux, uy):
        """Eq. (3) (and Eq. (18) for T) for all nine directions."""
        cu = self.cx * ux + self.cy * uy
        uu = ux * ux + uy * uy
        return self.w * rho * (1 + cu / CS2 + (cu * cu - CS2 * uu) / (2 * CS2 * CS2))

    def pull(self, fs, g_s, t_bottom):
        """Streaming of post-collision populations with the wall rules."""
        ly = self.ly
        t_top = self.p["t_top"]
        fa, fb, g = [], [], []
        for i in range(9):
            cx, cy = CX[i], CY[i]
            o = OPP[i]
            # source row of each destination row: y - cy; shift in x by cx
            def shifted(a):
                a = torch.roll(a, shifts=cx, dims=-1)
                if cy == 1:
                    return torch.cat([a[..., :1, :] * 0, a[..., :-1, :]], dim=-2)
                if cy == -1:
                    return torch.cat([a[..., 1:, :], a[..., :1, :] * 0], dim=-2)
                return a
            sa, sb, sg = shifted(fs[0][i]), shifted(fs[1][i]), shifted(g_s[i])
            if cy != 0:
                wall_row = 0 if cy == 1 else ly - 1
                mask = torch.zeros(ly, 1, dtype=torch.float64)
                mask[wall_row] = 1.0
                # bounce-back at the wall row: own post-collision opposite value
                sa = sa * (1 - mask) + fs[0][o] * mask
                sb = sb * (1 - mask) + fs[1][o] * mask
                if cy == 1:
                    # solid source below, at the column x - cx
                    tw = torch.roll(t_bottom, shifts=cx, dims=0).view(1, -1)
                else:
                    tw = torch.full((1, self.lx), t_top, dtype=torch.float64)
                sg = sg * (1 - mask) + (2 * W[i] * tw - g_s[o]) * mask
            fa.append(sa)
            fb.append(sb)
            g.append(sg)
        return torch.stack(fa), torch.stack(fb), torch.stack(g)

    def padded(self, field, wall):
        """Field with two ghost rows at the wall value below and above."""
        ghost = torch.full((2, self.lx), float(wall), dtype=torch.float64)
        return torch.cat([ghost, field, ghost], dim=0)

    def stencil_sum(self, padded, radius, weight):
        """sum_c weight(|c|^2) psi(x + c) c over the (2r+1)^2 square."""
        sx = torch.zeros(self.ly, self.lx, dtype=torch.float64)
        sy = torch.zeros(self.ly, self.lx, dtype=torch.float64)
        for dy in range(-radius, radius + 1):
            for dx in range(-radius, radius + 1):
                wgt = weight(dx * dx + dy * dy)
                if wgt == 0.0 or (dx == 0 and dy == 0):
                    continue
                v = torch.roll(padded[2 + dy:2 + dy + self.ly], shifts=-dx, dims=-1)
                sx = sx + wgt * v * dx
                sy = sy + wgt * v * dy
        return sx, sy

    def macroscopic(self, fa, fb, g):
        """Moments, forces and velocities of pre-collision populations."""
        p = self.p
        rho0 = p["rho0"]
        ra, rb, temp = fa.sum(0), fb.sum(0), g.sum(0)
        jx = (self.cx * (fa + fb)).sum(0)
        jy = (self.cy * (fa + fb)).sum(0)
        rw = p["rho_wall"]
        psx = [self.padded(r / rho0, rw[k] / rho0) for k, r in enumerate((ra, rb))]
        pss = [self.padded(rho0 * (1 - torch.exp(-r / rho0)), rho0 * (1 - math.exp(-rw[k] / rho0)))
               for k, r in enumerate((ra, rb))]
        forces = []
        for l, rl in enumerate((ra, rb)):
            m = 1 - l
            cx_, cy_ = self.stencil_sum(psx[m], 1, _w_weight)
            ax, ay = self.stencil_sum(pss[l], 1, _w_weight)
            qx, qy = self.stencil_sum(pss[l], 2, _p_weight)
            here_x = rl / rho0
            here_s = rho0 * (1 - torch.exp(-rl / rho0))
            fx = -p["g12"] * here_x * cx_ - here_s * (p["g_a"][l] * ax + p["g_r"][l] * qx)
            fy = -p["g12"] * here_x * cy_ - here_s * (p["g_a"][l] * ay + p["g_r"][l] * qy)
            fy = fy + rl * p["alpha_g"] * temp
            forces.append((fx, fy))
        rho = ra + rb
        ux, uy = jx / rho, jy / rho
        Fx = forces[0][0] + forces[1][0]
        Fy = forces[0][1] + forces[1][1]
        hx, hy = ux + Fx / (2 * rho), uy + Fy / (2 * rho)
        return dict(ra=ra, rb=rb, temp=temp, ux=ux, uy=uy, forces=forces, hx=hx, hy=hy)

    def collide(self, fa, fb, g, m):
        p = self.p
        tau, tau_g = p["tau"], p["tau_g"]
        out = []
        for l, (f, rl) in enumerate(((fa, m["ra"]), (fb, m["rb"]))):
            fx, fy = m["forces"][l]
            ulx, uly = m["ux"] + tau * fx / rl, m["uy"] + tau * fy / rl
            out.append(f - (f - self.equilibrium(rl, ulx, uly)) / tau)
        gs = g - (g - self.equilibrium(m["temp"], m["hx"], m["hy"])) / tau_g
        return out[0], out[1], gs

    # ---------------------------------------------------------------- API
    def initial_state(self, rho_a, rho_b, temp):
        """f*(0): collision of the rest equilibria of the given fields."""
        z = torch.zeros_like(rho_a)
        fa, fb, g = (self.equilibrium(rho_a, z, z), self.equilibrium(rho_b, z, z),
                     self.equilibrium(temp, z, z))
        m = self.macroscopic(fa, fb, g)
        return self.collide(fa, fb, g, m)

    def step(self, state, t_bottom):
        """f*(t) -> (f*(t+1), pre-collision f(t+1), macroscopic of t+1)."""
        fa, fb, g = self.pull((state[0], state[1]), state[2], t_bottom)
        m = self.macroscopic(fa, fb, g)
        return self.collide(fa, fb, g, m), (fa, fb, g), m

    def nu_top(self, g_pre):
        """Top-wall Nusselt number of pre-collision temperature populations."""
        t_row = g_pre.sum(0)[self.ly - 1]
        return 2 * self.ly / self.p["dt_nominal"] * (t_row - self.p["t_top"]).mean()

    def loss(self, state0, t_bottom, nsteps):
        """Time average over t = 1..nsteps of Nu_top(t)."""
        state = state0
        total = torch.zeros((), dtype=torch.float64)
        for _ in range(nsteps):
            state, pre, _ = self.step(state, t_bottom)
            total = total + self.nu_top(pre[2])
        return total / nsteps
