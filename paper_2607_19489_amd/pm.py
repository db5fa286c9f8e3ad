"""Particle-mesh time loop around the solver (the binary-orbit workload).

Argument marshalling and loop orchestration only: the hierarchy that tracks
the particles is built by the library on the host, deposition, interpolation
and the leapfrog updates run as HIP kernels, forces come from afmm_solve.

One step of the kick-drift-kick leapfrog with fixed dt (Sec. 4, Fig.
fig:binary: a fixed time step keeps the integrator symplectic):
    v += dt/2 a(x);  x += dt v;  [re-plan if the grid around x changed];  v += dt/2 a(x)
with a(x) = CIC interpolation of the solver's cell accelerations, the cell
masses being the CIC deposit of the particles at the finest level.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np
import torch

from ._lib import HierarchyC, check, lib
from .afmm import Plan, _stream_handle


class ParticleHierarchy:
    """A graded hierarchy refined around particles (afmm_particle_hierarchy_create),
    copied into arrays with the interface Plan expects."""

    def __init__(self, pos: np.ndarray, levelmin: int, levelmax: int, nexpand: int = 2, boxlen: float = 1.0):
        pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
        h = C.c_void_p()
        check(lib().afmm_particle_hierarchy_create(levelmin, levelmax, nexpand, pos.shape[0],
                                                   pos.ctypes.data_as(C.c_void_p), boxlen, C.byref(h)),
              "afmm_particle_hierarchy_create")
        try:
            v = HierarchyC()
            check(lib().afmm_particle_hierarchy_view(h, C.byref(v)), "afmm_particle_hierarchy_view")
            self.levelmin, self.levelmax = int(v.levelmin), int(v.levelmax)
            nl = self.levelmax - self.levelmin + 1
            self.ncell = np.ctypeslib.as_array(v.ncell, shape=(nl,)).copy()
            total = int(self.ncell.sum())
            self._ijk = np.ctypeslib.as_array(v.ijk, shape=(3 * total,)).copy().reshape(-1, 3)
            self._ref = np.ctypeslib.as_array(v.refined, shape=(total,)).copy()
        finally:
            lib().afmm_particle_hierarchy_destroy(h)
        self.boxlen = boxlen
        self.total = total

    def flat_ijk(self):
        return self._ijk

    def flat_refined(self):
        return self._ref

    def leaf_mask(self):
        return self._ref == 0

    def level_of(self):
        return np.repeat(np.arange(self.levelmin, self.levelmax + 1, dtype=np.int32), self.ncell)

    def same_as(self, other: "ParticleHierarchy") -> bool:
        return (other is not None and self.levelmin == other.levelmin and self.levelmax == other.levelmax
                and np.array_equal(self.ncell, other.ncell) and np.array_equal(self._ijk, other._ijk)
                and np.array_equal(self._ref, other._ref))


def cic_deposit(plan: Plan, level: int, pos: torch.Tensor, pmass: torch.Tensor, cell_mass: torch.Tensor,
                stream: Optional[torch.cuda.Stream] = None):
    check(lib().afmm_cic_deposit(plan.handle, level, pos.shape[0], C.c_void_p(pos.data_ptr()),
                                 C.c_void_p(pmass.data_ptr()), C.c_void_p(cell_mass.data_ptr()),
                                 _stream_handle(stream)), "afmm_cic_deposit")
    return cell_mass


def cic_interpolate(plan: Plan, level: int, pos: torch.Tensor, cell_acc: torch.Tensor,
                    cell_phi: Optional[torch.Tensor] = None, stream: Optional[torch.cuda.Stream] = None):
    n = pos.shape[0]
    acc = torch.empty(n, 3, dtype=torch.float64, device=pos.device)
    phi = torch.empty(n, dtype=torch.float64, device=pos.device) if cell_phi is not None else None
    check(lib().afmm_cic_interpolate(plan.handle, level, n, C.c_void_p(pos.data_ptr()),
                                     C.c_void_p(cell_acc.data_ptr()),
                                     C.c_void_p(cell_phi.data_ptr()) if cell_phi is not None else None,
                                     C.c_void_p(acc.data_ptr()), C.c_void_p(phi.data_ptr()) if phi is not None else None,
                                     _stream_handle(stream)), "afmm_cic_interpolate")
    return acc, phi


def update(state: torch.Tensor, rate: torch.Tensor, dt: float, stream: Optional[torch.cuda.Stream] = None):
    """state += dt * rate (contiguous float64 device tensors of equal size)."""
    check(lib().afmm_particles_update(state.numel(), dt, C.c_void_p(rate.data_ptr()), C.c_void_p(state.data_ptr()),
                                      _stream_handle(stream)), "afmm_particles_update")
    return state


class ParticleMesh:
    """Kick-drift-kick leapfrog of particles whose forces come from the FMM on a
    hierarchy that follows them (re-planned whenever the grid around them changes)."""

    def __init__(self, pos, vel, mass, levelmin: int, levelmax: int, nexpand: int = 2, p: int = 6,
                 precision: str = "fp64", G: float = 1.0, boxlen: float = 1.0, **plan_kw):
        self.pos = torch.as_tensor(np.asarray(pos, dtype=np.float64)).cuda().contiguous()
        self.vel = torch.as_tensor(np.asarray(vel, dtype=np.float64)).cuda().contiguous()
        self.mass = torch.as_tensor(np.asarray(mass, dtype=np.float64)).cuda().contiguous()
        self.levelmin, self.levelmax, self.nexpand = levelmin, levelmax, nexpand
        self.p, self.precision, self.G, self.boxlen, self.plan_kw = p, precision, G, boxlen, plan_kw
        self.h: Optional[ParticleHierarchy] = None
        self.plan: Optional[Plan] = None
        self._cells: Optional[np.ndarray] = None
        self.replans = 0
        self.t = 0.0
        self.acc, self.phi = self._forces()

    def _cloud_cells(self, pos: np.ndarray) -> np.ndarray:
        """Cloud cells floor(x 2^l / boxlen - 1/2) of every particle at every level
        the hierarchy builder refines (levelmin .. levelmax - 1), in the builder's
        own arithmetic (one product and one difference in double precision): the
        particles' hierarchy depends on their positions through these alone."""
        inv_h = np.array([float(1 << int(l)) / self.boxlen for l in range(self.levelmin, self.levelmax)])
        return np.floor(pos[None, :, :] * inv_h[:, None, None] - 0.5).astype(np.int64)

    def _ensure_plan(self):
        pos = self.pos.cpu().numpy()
        cells = self._cloud_cells(pos)
        if self.h is not None and self._cells is not None and np.array_equal(cells, self._cells):
            return  # no cloud moved to another cell: same hierarchy, same plan
        h = ParticleHierarchy(pos, self.levelmin, self.levelmax, self.nexpand, self.boxlen)
        self._cells = cells
        if h.same_as(self.h):
            return
        if self.plan is not None:
            self.plan.close()
        self.h = h
        self.plan = Plan(h, p=self.p, precision=self.precision, G=self.G, boxlen=self.boxlen, **self.plan_kw)
        self.cell_mass = torch.zeros(h.total, dtype=torch.float64, device="cuda")
        self.cell_phi = torch.zeros(h.total, dtype=torch.float64, device="cuda")
        self.cell_acc = torch.zeros(h.total, 3, dtype=torch.float64, device="cuda")
        self.replans += 1

    def _forces(self):
        """Accelerations and potentials at the particles for the current positions."""
        self._ensure_plan()
        lev = self.h.levelmax
        cic_deposit(self.plan, lev, self.pos, self.mass, self.cell_mass)
        self.plan.solve(self.cell_mass, phi=self.cell_phi, acc=self.cell_acc)
        return cic_interpolate(self.plan, lev, self.pos, self.cell_acc, self.cell_phi)

    def step(self, dt: float):
        update(self.vel, self.acc, 0.5 * dt)
        update(self.pos, self.vel, dt)
        self.acc, self.phi = self._forces()
        update(self.vel, self.acc, 0.5 * dt)
        self.t += dt

    def energy(self) -> dict:
        """Kinetic energy and the particles' potential energy 1/2 sum m phi(x) (the
        latter includes each cloud's constant self part)."""
        m = self.mass
        ke = 0.5 * float((m[:, None] * self.vel * self.vel).sum())
        pe = 0.5 * float((m * self.phi).sum())
        return {"kinetic": ke, "potential": pe, "total": ke + pe}

    def close(self):
        if self.plan is not None:
            self.plan.close()
            self.plan = None


def binary_initial(G: float = 1.0, gm: float = 0.01, sep: float = 0.15, centre=(0.5, 0.5, 0.5)):
    """Two equal masses (G m = gm each) on a circular orbit of separation `sep`
    about `centre` in the x-y plane (Sec. 4, Fig. fig:binary): positions,
    velocities, masses and the angular velocity of the orbit."""
    m = gm / G
    omega = np.sqrt(2.0 * gm / sep ** 3)
    r = 0.5 * sep
    c = np.asarray(centre, dtype=np.float64)
    pos = np.array([c + [r, 0, 0], c - [r, 0, 0]])
    vel = np.array([[0, omega * r, 0], [0, -omega * r, 0]], dtype=np.float64)
    return pos, vel, np.array([m, m]), omega
