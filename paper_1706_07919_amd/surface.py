"""Surface buffers of one or more scatterers on the device.

The per-body icosphere comes from the library's host mesh builder
(``bem_mesh_icosphere``); bodies are concatenated in order (the surface S of
Eq. BRIEF is the union of the scatterer surfaces) and uploaded once.
"""
from __future__ import annotations

import numpy as np

from . import native


def host_surface(bodies, rescale_area: bool = True):
    """(x, nrm, w, bc) host arrays of the concatenated bodies.  ``bodies`` are
    objects with center, radius, aspect, level, bc attributes."""
    xs, ns, ws, bs = [], [], [], []
    for b in bodies:
        x, n, w, _ = native.bem_mesh_icosphere(b.level, b.radius, b.aspect, b.center, rescale_area)
        xs.append(x); ns.append(n); ws.append(w)
        bs.append(np.full(x.shape[0], b.bc, dtype=np.uint8))
    return np.concatenate(xs), np.concatenate(ns), np.concatenate(ws), np.concatenate(bs)


class DeviceSurface:
    """Device copies of nodes, normals, weights and BC flags plus the C struct."""

    def __init__(self, x, nrm, w, bc, device="cuda"):
        import torch
        self.n = int(x.shape[0])
        self.x = torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64).to(device)
        self.nrm = torch.as_tensor(np.ascontiguousarray(nrm), dtype=torch.float64).to(device)
        self.w = torch.as_tensor(np.ascontiguousarray(w), dtype=torch.float64).to(device)
        self.bc = torch.as_tensor(np.ascontiguousarray(bc), dtype=torch.uint8).to(device)
        self.struct = native.surface_struct(self.n, self.x, self.nrm, self.w, self.bc)

    @classmethod
    def from_bodies(cls, bodies, rescale_area=True, device="cuda"):
        return cls(*host_surface(bodies, rescale_area), device=device)


class DeviceQuadSurface:
    """Six-node elements of one body on the device (nodes, normals, BC flags,
    element table) plus the C struct; the mesh comes from the library's host
    builder (``bem_mesh_quadratic``)."""

    def __init__(self, x, nrm, bc, elems, device="cuda"):
        import torch
        self.n = int(x.shape[0])
        self.n_elem = int(elems.shape[0])
        self.x = torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64).to(device)
        self.nrm = torch.as_tensor(np.ascontiguousarray(nrm), dtype=torch.float64).to(device)
        self.bc = torch.as_tensor(np.ascontiguousarray(bc), dtype=torch.uint8).to(device)
        self.elem = torch.as_tensor(np.ascontiguousarray(elems), dtype=torch.int32).to(device)
        self.struct = native.quad_surface_struct(self.n, self.x, self.nrm, self.bc, self.n_elem,
                                                 self.elem)

    @classmethod
    def from_body(cls, body, nu, device="cuda"):
        """``body``: center, radius, aspect, bc (its level is not used)."""
        x, nrm, elems = native.bem_mesh_quadratic(nu, body.radius, body.aspect, body.center)
        bc = np.full(x.shape[0], body.bc, dtype=np.uint8)
        return cls(x, nrm, bc, elems, device=device)
