"""One-system NPT molecular dynamics on the device: real-space pairs
(rbe_real_*), the random batch Ewald Fourier part (rbe_*), and the Langevin
NPT integrator (rbe_md_*), in the order of section 3.3 (forces and pressure
between the two halves of the step).  Orchestration only: every step of the
computation is a kernel of librbe.so.
"""

import numpy as np

from .rbe import RBE, Integrator, RealSpace


class NPTSystem:
    """Positions, momenta and forces resident on the GPU between steps.

    sysd: dict with pos (N,3), q, mass, box; alpha, p, coulomb;
    md: dict with dt, kT, p_ext, gamma_p, gamma_cell, mass_cell, mass_cell_z,
        ftm, box_mode ('iso', 'semiiso' or 'aniso'), rc; optional types + lj for the
        real-space Lennard-Jones term; optional rigid = dict(first, count,
        d_oh, d_hh) for rigid 3-site molecules (whole, not split by the
        periodic boundary); optional skin (> 0: real-space neighbour lists);
        optional sampler ('exact' or 'mh', with mh_iters moves per step);
        optional fused (True: the Fourier step as one launch, False: two
        launches, the default; see RBE.set_fused).
    """

    def __init__(self, sysd, md, precision="fp32", seed=0, system_id=0, momenta=None,
                 stream=None, device="cuda:0", real_precision="fp64"):
        import torch
        self.torch = torch
        dev = torch.device(device)
        t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
        self.n = len(sysd["q"])
        pos = np.asarray(sysd["pos"], dtype=np.float64)
        self.x, self.y, self.z = (t(pos[:, a]) for a in range(3))
        mass = np.asarray(sysd["mass"], dtype=np.float64)
        if momenta is None:
            momenta = np.zeros((self.n, 3))
        self.px, self.py, self.pz = (t(momenta[:, a]) for a in range(3))
        self.f = [torch.zeros(self.n, dtype=torch.float64, device=dev) for _ in range(3)]
        self.vk = torch.zeros(6, dtype=torch.float64, device=dev)
        self.vr = torch.zeros(6, dtype=torch.float64, device=dev)
        self.ek = torch.zeros(1, dtype=torch.float64, device=dev)
        self.er = torch.zeros(1, dtype=torch.float64, device=dev)
        q = t(sysd["q"])
        mode = md.get("box_mode", "iso")
        b = [float(v) for v in sysd["box"]]
        # the Fourier part only checks the cell's shape: a non-cubic cell under
        # isotropic coupling is a general rectangular one there
        kmode = "aniso" if mode == "iso" and not (b[0] == b[1] == b[2]) else mode
        self.kspace = RBE(q, sysd["box"], sysd["p"], sysd["alpha"], coulomb=sysd["coulomb"],
                          precision=precision, box_mode=kmode, seed=seed, system_id=system_id,
                          stream=stream)
        if md.get("sampler", "exact") != "exact":
            self.kspace.set_sampler(md["sampler"], int(md.get("mh_iters", 1)))
        if md.get("fused") is not None:
            self.kspace.set_fused(1 if md["fused"] else 0)
        types = None
        if md.get("lj") is not None:
            types = torch.tensor(np.asarray(md["types"], dtype=np.int32), device=dev)
        self.real = RealSpace(q, sysd["box"], sysd["alpha"], md["rc"], coulomb=sysd["coulomb"],
                              types=types, lj=md.get("lj"), stream=stream,
                              precision=real_precision)
        if md.get("skin", 0.0) > 0.0:
            self.real.set_skin(md["skin"])
        self.integ = Integrator(t(mass), sysd["box"], md["dt"], md["kT"], md["p_ext"],
                                md["gamma_p"], md["gamma_cell"], md["mass_cell"],
                                md.get("mass_cell_z", 0.0), box_mode=mode, ftm=md["ftm"],
                                seed=seed, system_id=system_id, stream=stream)
        rg = md.get("rigid")
        if rg:
            self.integ.set_rigid(rg["first"], rg["count"], rg["d_oh"], rg["d_hh"])
        self.step_index = 0
        self._box_ptr = None
        self._forces(sample_step=2**63, first=True)
        self.integ.pressure(self.x, self.y, self.z, self.px, self.py, self.pz, *self.f,
                            self.vk, self.vr)

    def _forces(self, sample_step, first=False):
        self.kspace.sample_k(sample_step)
        self.kspace.forces_pressure(self.x, self.y, self.z, *self.f, accumulate=False,
                                    virial6=self.vk, energy=self.ek)
        self.real.forces(self.x, self.y, self.z, *self.f, accumulate=True, virial6=self.vr,
                         energy=self.er)

    def _bind_device_box(self):
        # the integrator's mid-step cell feeds both force evaluations
        if self._box_ptr is None:
            self._box_ptr = self.integ.box_dev_ptr()
            self.real.set_box_dev_ptr(self._box_ptr)
        self.kspace.rescale_box_dev_ptr(self._box_ptr)

    def step(self, nsteps=1):
        for _ in range(nsteps):
            s = self.step_index
            self.integ.first_half(s, self.x, self.y, self.z, self.px, self.py, self.pz, *self.f)
            self._bind_device_box()
            self._forces(sample_step=s)
            self.integ.second_half(self.x, self.y, self.z, self.px, self.py, self.pz, *self.f,
                                   self.vk, self.vr)
            self.step_index += 1

    def state(self):
        st = self.integ.state()
        st["pos"] = np.stack([a.cpu().numpy() for a in (self.x, self.y, self.z)], 1)
        st["mom"] = np.stack([a.cpu().numpy() for a in (self.px, self.py, self.pz)], 1)
        return st

    def check(self):
        self.kspace.check()
        self.real.check()
        self.integ.check()
