"""Seeded cases shared by the GPU tests: geometry from the oracle, inputs from
the workload generator, the same numbers handed to both sides."""
import numpy as np

from oracle import geometry as geo
from oracle import letkf as ol
from oracle import philox
from paper_1408_7069_amd import workload as wl


class Case:
    def __init__(self, N, eps, b, h, m, seed=0, taper_c=0.0, rho=1.05, a=0.99, sigma=0.1,
                 r0=0.15, pitch=0.5, fp64=False, r_scale=1.0, bank_screens=8, piston=False):
        self.N, self.eps, self.b, self.h, self.m = N, eps, b, h, m
        self.rng = np.random.default_rng(seed)
        self.G = geo.geometry_for(N, eps)
        self.doms = geo.domains(self.G, b, h)
        self.prm = ol.Params(a=a, rho=rho, r_scale=r_scale, b=b, h=h, taper_c=taper_c, piston=piston)
        self.noise_scale = np.sqrt(1 - a * a)   # AR(1) model noise, fixed at construction
        self.sigma, self.r0, self.pitch, self.fp64 = sigma, r0, pitch, fp64
        self.ij = self.G.node_coords()
        self.r = np.full(self.G.n_slopes, sigma * sigma) * self.rng.uniform(0.8, 1.25, self.G.n_slopes)
        side = 1
        while side < 2 * (N + 1):
            side *= 2
        self.bank = wl.noise_bank(bank_screens, side, pitch, r0, 25.0, a, self.rng)
        self.seed = int(self.rng.integers(1, 2 ** 62))
        self.dt = np.float64 if fp64 else np.float32

    def spec(self, B, **kw):
        d = dict(n_sub=self.N, m=self.m, domain_size=self.b, halo=self.h,
                 obscuration=0.0 if self.eps is None else self.eps,
                 mask=geo.square_mask(self.N) if self.eps is None else None,
                 rho=self.prm.rho, r_diag=self.r, r_scale=self.prm.r_scale, ar_coeff=self.prm.a,
                 taper_c=self.prm.taper_c, noise_bank=self.bank, seed=self.seed,
                 precision=B.FP64 if self.fp64 else B.FP32, piston=self.prm.piston)
        d.update(kw)
        return B.InstanceSpec(**d)

    def noise(self, scale=1.0):
        """An explicit V (n, m): von Karman screens sampled at the nodes."""
        G = 2 * (self.N + 1)
        s = wl.vk_screens(G, self.pitch, self.r0, 25.0, self.m, self.rng)
        V = np.stack([x[self.ij[:, 0], self.ij[:, 1]] for x in s], axis=1)
        return (scale * self.noise_scale * V).astype(self.dt)

    def truth(self):
        s = wl.vk_screens(2 * (self.N + 1), self.pitch, self.r0, 25.0, 1, self.rng)[0]
        return s[self.ij[:, 0], self.ij[:, 1]]

    def slopes(self, truth):
        y = geo.apply_slopes(self.G, truth) + wl.gaussian_noise(self.G.n_slopes, self.sigma, self.rng)
        return y.astype(self.dt)

    def bank_V(self, frame, instance=0):
        return philox.bank_noise(self.bank, self.ij, self.m, self.seed, instance, frame)

    def oracle_analysis(self, Xb, y, **kw):
        """The analysis (and the piston removal when the case has it on)."""
        Xa = ol.analysis(self.G, self.doms, np.asarray(Xb, np.float64), np.asarray(y, np.float64),
                         self.r, self.prm, **kw)
        if self.prm.piston:
            from oracle import piston
            Xa = piston.remove(self.G, self.doms, Xa, y)
        return Xa


def rel_err(got, ref):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))
