"""One SIMP iteration and a SIMP trajectory, in the order of the Workflow section:
finite-element analysis, sensitivity computation, sensitivity filtering, OC
design update, convergence measure.

Density-filter mode (the default):
  xPhys = filter(x) with the passive reset; E = Emin + xPhys^p (E0 - Emin);
  K(E) u = f; c = f^T u; dc = -p xPhys^(p-1)(E0 - Emin) u_e^T KE u_e;
  dc~ = H (dc_D / Hs); dv~ = w^D; the OC multiplier makes the design-element sum
  of filter(x_new) equal to volfrac * (number of design elements).
  With ``vol_mode == "all"`` the sum runs over every element instead (passive
  solids at 1, voids at 0) and equals volfrac * nel.
Sensitivity-filter mode (the filter the paper's text describes):
  xPhys = x; dc~ = H(x dc)/(Hs max(1e-3, x)); dv = 1; volume = sum of x over
  design elements.
``change`` = max |x_new - x|.
"""

from __future__ import annotations

import numpy as np

from . import fem, filt, oc
from .ke import element_stiffness


class SimpOracle:
    def __init__(self, p, solver=None):
        self.p = p
        self.KE = element_stiffness(p.nu)
        self.edof = fem.element_dofs(p.nelx, p.nely, p.nelz)
        self.mask = np.zeros(p.nel, np.int8) if p.mask is None else np.asarray(p.mask, np.int8)
        self.filter = filt.Filter(p.nelx, p.nely, p.nelz, p.rmin, self.mask)
        self.design = self.mask == 0
        self.n_design = int(self.design.sum())
        if getattr(p, "vol_mode", "design") == "all":
            # every element counts (fixed solids as 1, fixed voids as 0) against
            # volfrac * nel; the design elements carry what the solids leave
            self.target = p.volfrac * p.nel - int((self.mask == 2).sum())
        else:
            self.target = p.volfrac * self.n_design
        if p.filter_mode == "density":
            self.w = self.filter.volume_weights()
        else:
            self.w = self.design.astype(float)
        self.solver = solver

    # -- pieces -----------------------------------------------------------
    def physical(self, x):
        if self.p.filter_mode == "density":
            return self.filter.forward(x)
        xp = x.copy()
        xp[self.mask == 1] = 0.0
        xp[self.mask == 2] = 1.0
        return xp

    def volume(self, x):
        """Plain volume measure: design-element sum of the physical density."""
        return float(self.physical(x)[self.design].sum())

    def solve(self, E):
        p = self.p
        if self.solver is not None:
            return self.solver(E)
        K = fem.assemble(E, self.KE, self.edof, p.ndof)
        return fem.solve(K, p.f, p.fixed_dofs)

    def step(self, x, lam_mode="exact", oc_tol=1e-12):
        p = self.p
        xphys = self.physical(x)
        E = fem.simp_modulus(xphys, p.E0, p.Emin, p.penal)
        u = self.solve(E)
        ce = fem.element_energy(self.KE, self.edof, u)
        c = fem.compliance(p.f, u)
        dc = fem.compliance_sensitivity(xphys, ce, p.E0, p.Emin, p.penal)
        if p.filter_mode == "density":
            dcf = self.filter.adjoint(dc)
            dvf = self.w.copy()
        else:
            dcf = self.filter.sensitivity(x, dc)
            dvf = np.ones_like(x)
        if lam_mode == "exact":
            xnew, lam = oc.oc_exact(x, dcf, dvf, self.w, self.target, p.move, p.eta, self.design)
        else:
            xnew, lam, _ = oc.oc_bisection(x, dcf, dvf, self.volume, self.target, p.move, p.eta,
                                           self.design, tol=oc_tol)
        return {
            "xphys": xphys, "E": E, "u": u, "ce": ce, "c": c, "dc": dc, "dcf": dcf,
            "dvf": dvf, "x_new": xnew, "lam": lam,
            "change": float(np.max(np.abs(xnew - x))) if x.size else 0.0,
            "volume": self.volume(xnew),
        }

    def trajectory(self, n_iter=None, x0=None, keep=False):
        p = self.p
        x = p.initial_design() if x0 is None else x0.copy()
        hist = []
        for _ in range(p.n_iter if n_iter is None else n_iter):
            r = self.step(x)
            rec = {k: r[k] for k in ("c", "lam", "change", "volume")}
            if keep:
                rec["x"] = x.copy()
                rec["x_new"] = r["x_new"].copy()
            hist.append(rec)
            x = r["x_new"]
        return x, hist
