"""ctypes binding of include/drpf.h with torch-owned device memory.

Names follow the C API: ``Grid`` wraps a drpf_grid handle plus its workspace tensor;
``DeviceState`` owns the state tensors and the drpf_state struct that points at them.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(HERE, "libdrpf.so")

DRPF_OK, DRPF_EINVAL, DRPF_EWORKSPACE, DRPF_EHIP, DRPF_ENONFINITE, DRPF_EUNSUPPORTED = range(6)
LOCATIONS = {"center": 0, "face_x": 1, "face_y": 2, "face_z": 3, "edge_xy": 4, "edge_xz": 5,
             "edge_yz": 6}
BCS = {"neumann": 0, "dirichlet": 1, "face_dirichlet": 2}
NKERNELS = 19
OBSERVABLES = ("mass", "wetted_radius", "centroid_height", "kinetic_energy", "max_div")


class DrpfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"drpf error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lz", ctypes.c_double),
        ("re", ctypes.c_double), ("ca", ctypes.c_double), ("cn", ctypes.c_double),
        ("pe", ctypes.c_double), ("wi", ctypes.c_double), ("beta", ctypes.c_double),
        ("theta_bottom_deg", ctypes.c_double), ("theta_top_deg", ctypes.c_double),
        ("rho_ratio", ctypes.c_double), ("mu_ratio", ctypes.c_double),
        ("dt", ctypes.c_double), ("s_factor", ctypes.c_double),
        ("a_ext", ctypes.c_double * 3),
        ("viscoelastic", ctypes.c_int), ("precision", ctypes.c_int),
        ("constitutive", ctypes.c_int), ("giesekus_alpha", ctypes.c_double),
        ("refine", ctypes.c_int), ("advection", ctypes.c_int), ("d_w", ctypes.c_double),
        ("u_wall_bottom", ctypes.c_double * 2), ("u_wall_top", ctypes.c_double * 2),
        ("check_finite_every", ctypes.c_int),
    ]


FIELDS = ("phi", "u", "v", "w", "p", "tau", "theta")


class FieldLayout(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int * 3), ("stride", ctypes.c_size_t * 3), ("elems", ctypes.c_size_t),
        ("arrays", ctypes.c_int), ("origin", ctypes.c_double * 3), ("spacing", ctypes.c_double * 3),
    ]


class Layout(ctypes.Structure):
    _fields_ = [("elem_bytes", ctypes.c_int), ("field", FieldLayout * len(FIELDS)),
                ("state_bytes", ctypes.c_size_t)]


class State(ctypes.Structure):
    _fields_ = [
        ("phi", ctypes.c_void_p * 3),
        ("u", ctypes.c_void_p * 2), ("v", ctypes.c_void_p * 2), ("w", ctypes.c_void_p * 2),
        ("p", ctypes.c_void_p * 2),
        ("tau", (ctypes.c_void_p * 6) * 2),
        ("step", ctypes.c_longlong),
        ("theta", ctypes.c_void_p * 6),
    ]


class Adj(ctypes.Structure):
    _fields_ = [
        ("phi", ctypes.c_void_p * 2),
        ("u", ctypes.c_void_p * 2), ("v", ctypes.c_void_p * 2), ("w", ctypes.c_void_p * 2),
        ("p", ctypes.c_void_p * 2),
        ("tau", (ctypes.c_void_p * 6) * 2),
    ]


_LIB = None


def lib():
    """Loads libdrpf.so once. Raises if it has not been built: there is no fallback."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(lib_path):
            raise RuntimeError(f"{lib_path} not found: build it with "
                               "`python -m paper_2111_04577_amd.build_lib`")
        L = ctypes.CDLL(lib_path)
        vp, i, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
        P = ctypes.POINTER
        sig = {
            "drpf_params_default": [P(Params)],
            "drpf_validate": [P(Params)],
            "drpf_field_elems": [P(Params), P(sz), P(sz)],
            "drpf_workspace_bytes": [P(Params), P(sz)],
            "drpf_init_grid": [P(Params), vp, sz, vp, P(vp)],
            "drpf_destroy": [vp],
            "drpf_step": [vp, P(State), i, vp],
            "drpf_prolong": [vp, vp, vp, vp, vp, vp, vp, vp],
            "drpf_restrict": [vp, vp, vp, i, vp],
            "drpf_helmholtz_solve": [vp, i, i, d, d, vp, vp, vp, vp],
            "drpf_helmholtz_solve_static": [vp, i, i, d, d, vp, vp, vp, vp],
            "drpf_state_layout": [vp, P(Layout)],
            "drpf_observables": [vp, P(State), P(d), i, vp],
            "drpf_debug_field": [vp, i, P(vp), P(sz)],
            "drpf_profile_begin": [vp, i, vp],
            "drpf_profile_end": [vp, P(d), P(i), i],
            "drpf_adjoint_workspace_bytes": [P(Params), P(sz)],
            "drpf_adjoint_attach": [vp, vp, sz],
            "drpf_adjoint_step": [vp, P(State), P(State), P(Adj), vp, vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.drpf_last_error.argtypes = []
        L.drpf_last_error.restype = ctypes.c_char_p
        L.drpf_kernel_name.argtypes = [ctypes.c_int]
        L.drpf_kernel_name.restype = ctypes.c_char_p
        _LIB = L
    return _LIB


def _check(rc):
    if rc != DRPF_OK:
        raise DrpfError(rc, lib().drpf_last_error().decode())


def make_params(cfg, precision=64) -> Params:
    """Params from any object with the drpf_params field names as attributes."""
    p = Params()
    lib().drpf_params_default(ctypes.byref(p))
    for name, _ in Params._fields_:
        if name in ("precision",):
            continue
        if hasattr(cfg, name):
            val = getattr(cfg, name)
            if name in ("a_ext", "u_wall_bottom", "u_wall_top"):
                getattr(p, name)[:] = [float(x) for x in val]
            else:
                setattr(p, name, val)
    p.precision = int(precision)
    return p


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class DeviceState:
    """State tensors on the device plus the drpf_state struct pointing at them.

    All arrays are views of one flat device buffer (three fine phi buffers, then u, v, w, p
    with two levels each, then the polymer stress when viscoelastic, then the log-conformation
    when the update takes that form), so a snapshot is one device copy."""

    def __init__(self, grid: "Grid", host: dict):
        import torch
        self.grid = grid
        dt = grid.torch_dtype
        dev = grid.device
        nf = int(np.prod(grid.fine_shape))
        nc = int(np.prod(grid.coarse_shape))
        ve = bool(grid.params.viscoelastic)
        lcr = grid.params.constitutive == 1
        ncoarse = 8 + (12 if ve else 0) + (6 if lcr else 0)
        self.flat = torch.empty(3 * nf + ncoarse * nc, dtype=dt, device=dev)
        views = []
        pos = 0
        for n, shape in [(nf, grid.fine_shape)] * 3 + [(nc, grid.coarse_shape)] * ncoarse:
            views.append(self.flat[pos:pos + n].view(shape))
            pos += n
        self.tensors = views
        t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=dt)
        self.phi = views[0:3]
        self.phi[0].copy_(t(host["phi"][0]))
        self.phi[1].copy_(t(host["phi"][1]))
        self.phi[2].zero_()
        for a, name in enumerate(("u", "v", "w", "p")):
            lv = views[3 + 2 * a:5 + 2 * a]
            for l in range(2):
                lv[l].copy_(t(host[name][l]))
            setattr(self, name, lv)
        if ve:
            self.tau = [views[11 + 6 * l:17 + 6 * l] for l in range(2)]
            for l in range(2):
                for m in range(6):
                    self.tau[l][m].copy_(t(host["tau"][l][m]))
        else:
            self.tau = None
        if lcr:
            self.theta = views[23:29]
            for m in range(6):
                self.theta[m].copy_(t(host["theta"][m]))
        else:
            self.theta = None
        self.c = State()
        self.c.step = int(host.get("step", 0))
        self._push()

    def _push(self):
        c = self.c
        for a in range(3):
            c.phi[a] = self.phi[a].data_ptr()
        for name in ("u", "v", "w", "p"):
            arr = getattr(c, name)
            for a in range(2):
                arr[a] = getattr(self, name)[a].data_ptr()
        if self.tau is not None:
            for lvl in range(2):
                for m in range(6):
                    c.tau[lvl][m] = self.tau[lvl][m].data_ptr()
        if self.theta is not None:
            for m in range(6):
                c.theta[m] = self.theta[m].data_ptr()

    def _pull(self):
        """Re-associate tensors with the pointers the library rotated."""
        by_ptr = {x.data_ptr(): x for x in self.tensors}
        c = self.c
        self.phi = [by_ptr[c.phi[a]] for a in range(3)]
        for name in ("u", "v", "w", "p"):
            arr = getattr(c, name)
            setattr(self, name, [by_ptr[arr[a]] for a in range(2)])
        if self.tau is not None:
            self.tau = [[by_ptr[c.tau[lvl][m]] for m in range(6)] for lvl in range(2)]

    def _offsets(self):
        base, es = self.flat.data_ptr(), self.flat.element_size()
        c = self.c
        offs = [(c.phi[a] - base) // es for a in range(3)]
        for name in ("u", "v", "w", "p"):
            arr = getattr(c, name)
            offs += [(arr[a] - base) // es for a in range(2)]
        if self.tau is not None:
            offs += [(c.tau[l][m] - base) // es for l in range(2) for m in range(6)]
        if self.theta is not None:
            offs += [(c.theta[m] - base) // es for m in range(6)]
        return offs

    @property
    def step(self) -> int:
        return int(self.c.step)

    def snapshot(self) -> dict:
        """One device copy of every buffer, with the current level assignment and step."""
        return {"flat": self.flat.clone(), "offsets": self._offsets(), "step": self.step}

    def restore(self, snap: dict):
        """Copies a snapshot back into this state's buffers (one device copy)."""
        self.flat.copy_(snap["flat"])
        base, es = self.flat.data_ptr(), self.flat.element_size()
        offs = iter(snap["offsets"])
        c = self.c
        for a in range(3):
            c.phi[a] = base + es * next(offs)
        for name in ("u", "v", "w", "p"):
            arr = getattr(c, name)
            for a in range(2):
                arr[a] = base + es * next(offs)
        if self.tau is not None:
            for l in range(2):
                for m in range(6):
                    c.tau[l][m] = base + es * next(offs)
        if self.theta is not None:
            for m in range(6):
                c.theta[m] = base + es * next(offs)
        c.step = int(snap["step"])
        self._pull()
        return self

    @staticmethod
    def struct_of(snap: dict, viscoelastic: bool) -> State:
        """A drpf_state over a snapshot's buffers (no copies); the snapshot must stay alive."""
        base, es = snap["flat"].data_ptr(), snap["flat"].element_size()
        offs = iter(snap["offsets"])
        c = State()
        for a in range(3):
            c.phi[a] = base + es * next(offs)
        for name in ("u", "v", "w", "p"):
            arr = getattr(c, name)
            for a in range(2):
                arr[a] = base + es * next(offs)
        if viscoelastic:
            for l in range(2):
                for m in range(6):
                    c.tau[l][m] = base + es * next(offs)
        c.step = int(snap["step"])
        return c

    def to_host(self) -> dict:
        """Copy to FP64 numpy arrays: {phi, u, v, w, p: [level n, level n-1], tau, step}."""
        h = lambda x: x.detach().double().cpu().numpy()
        out = {"phi": [h(self.phi[0]), h(self.phi[1])],
               "u": [h(a) for a in self.u], "v": [h(a) for a in self.v],
               "w": [h(a) for a in self.w], "p": [h(a) for a in self.p], "step": self.step}
        if self.tau is not None:
            out["tau"] = [[h(a) for a in self.tau[lvl]] for lvl in range(2)]
        else:
            z = np.zeros(self.grid.coarse_shape)
            out["tau"] = [[z.copy() for _ in range(6)] for _ in range(2)]
        if self.theta is not None:
            out["theta"] = [h(a) for a in self.theta]
        return out


class DeviceAdj:
    """Adjoint-state tensors (FP64, both levels) plus the drpf_adj struct pointing at them."""

    FIELDS = ("phi", "u", "v", "w", "p")

    def __init__(self, grid: "Grid", host: dict | None = None):
        import torch
        self.grid = grid
        dev = grid.device
        f64 = torch.float64
        shape = {"phi": grid.fine_shape}
        self.tensors = []

        def mk(name, arr=None):
            sh = shape.get(name, grid.coarse_shape)
            if arr is None:
                x = torch.zeros(sh, dtype=f64, device=dev)
            else:
                x = torch.as_tensor(np.ascontiguousarray(arr), dtype=f64, device=dev).contiguous().clone()
            self.tensors.append(x)
            return x

        for name in self.FIELDS:
            setattr(self, name, [mk(name, None if host is None else host[name][a]) for a in range(2)])
        if grid.params.viscoelastic:
            self.tau = [[mk("tau", None if host is None else host["tau"][lvl][m]) for m in range(6)]
                        for lvl in range(2)]
        else:
            self.tau = None
        self.c = Adj()
        self._push()

    def _push(self):
        for name in self.FIELDS:
            arr = getattr(self.c, name)
            for a in range(2):
                arr[a] = getattr(self, name)[a].data_ptr()
        if self.tau is not None:
            for lvl in range(2):
                for m in range(6):
                    self.c.tau[lvl][m] = self.tau[lvl][m].data_ptr()

    def _pull(self):
        by_ptr = {x.data_ptr(): x for x in self.tensors}
        for name in self.FIELDS:
            arr = getattr(self.c, name)
            setattr(self, name, [by_ptr[arr[a]] for a in range(2)])
        if self.tau is not None:
            self.tau = [[by_ptr[self.c.tau[lvl][m]] for m in range(6)] for lvl in range(2)]

    def to_host(self) -> dict:
        h = lambda x: x.detach().cpu().numpy()
        out = {name: [h(a) for a in getattr(self, name)] for name in self.FIELDS}
        if self.tau is not None:
            out["tau"] = [[h(a) for a in self.tau[lvl]] for lvl in range(2)]
        else:
            z = np.zeros(self.grid.coarse_shape)
            out["tau"] = [[z.copy() for _ in range(6)] for _ in range(2)]
        return out


class Grid:
    """One problem set-up on one device: the drpf_grid handle and its workspace tensor."""

    def __init__(self, cfg, precision=64, device="cuda:0", stream=None):
        import torch
        self.params = make_params(cfg, precision)
        L = lib()
        _check(L.drpf_validate(ctypes.byref(self.params)))
        nb = ctypes.c_size_t()
        _check(L.drpf_workspace_bytes(ctypes.byref(self.params), ctypes.byref(nb)))
        self.device = torch.device(device)
        self.torch_dtype = torch.float64 if precision == 64 else torch.float32
        # 256-byte alignment: torch's device allocator returns 512-byte aligned blocks
        self.workspace = torch.empty(int(nb.value) + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self._ws_ptr = base + off
        self.handle = ctypes.c_void_p()
        _check(L.drpf_init_grid(ctypes.byref(self.params), ctypes.c_void_p(self._ws_ptr),
                                ctypes.c_size_t(int(nb.value)), _stream_ptr(stream),
                                ctypes.byref(self.handle)))
        p = self.params
        r = 1 if p.refine == 1 else 2
        ry = 1 if p.ny == 1 else r
        self.fine_shape = (r * p.nz, ry * p.ny, r * p.nx)
        self.coarse_shape = (p.nz, p.ny, p.nx)

    def __del__(self):
        try:
            if getattr(self, "handle", None) and self.handle.value:
                lib().drpf_destroy(self.handle)
                self.handle = ctypes.c_void_p()
        except Exception:
            pass

    def state(self, host: dict) -> DeviceState:
        return DeviceState(self, host)

    def step(self, st: DeviceState, nsteps: int = 1, stream=None):
        """drpf_step. A failed finite check (check_finite_every > 0) raises DrpfError with code
        DRPF_ENONFINITE after the state has taken the steps up to and including the failed
        one (st.step says which)."""
        rc = lib().drpf_step(self.handle, ctypes.byref(st.c), int(nsteps), _stream_ptr(stream))
        st._pull()
        _check(rc)
        return st

    def layout(self) -> dict:
        """drpf_state_layout as {field: {n, stride, elems, arrays, origin, spacing}} plus
        elem_bytes and state_bytes."""
        L = Layout()
        _check(lib().drpf_state_layout(self.handle, ctypes.byref(L)))
        out = {"elem_bytes": L.elem_bytes, "state_bytes": int(L.state_bytes)}
        for f, name in enumerate(FIELDS):
            fl = L.field[f]
            out[name] = {"n": tuple(fl.n), "stride": tuple(int(x) for x in fl.stride), "elems": int(fl.elems),
                         "arrays": fl.arrays, "origin": tuple(fl.origin), "spacing": tuple(fl.spacing)}
        return out

    def attach_adjoint(self, stream=None):
        """Allocates and attaches the adjoint workspace (FP64 grids)."""
        import torch
        if getattr(self, "adj_workspace", None) is not None:
            return self
        L = lib()
        nb = ctypes.c_size_t()
        _check(L.drpf_adjoint_workspace_bytes(ctypes.byref(self.params), ctypes.byref(nb)))
        self.adj_workspace = torch.empty(int(nb.value) + 256, dtype=torch.uint8, device=self.device)
        base = self.adj_workspace.data_ptr()
        _check(L.drpf_adjoint_attach(self.handle, ctypes.c_void_p(base + (-base) % 256),
                                     ctypes.c_size_t(int(nb.value))))
        return self

    def adjoint(self, host: dict | None = None) -> DeviceAdj:
        return DeviceAdj(self, host)

    def adjoint_step(self, st, lam: DeviceAdj, grad3, next_state=None, stream=None):
        """One reverse step (drpf_adjoint_step): lam goes from the adjoint of step(st) to the
        adjoint of st; grad3 (device FP64 tensor of 3) is incremented. ``st`` and
        ``next_state`` (the state after the step, optional) are DeviceState objects or
        drpf_state structs."""
        c = st.c if isinstance(st, DeviceState) else st
        nxt = None
        if next_state is not None:
            nxt = ctypes.byref(next_state.c if isinstance(next_state, DeviceState) else next_state)
        _check(lib().drpf_adjoint_step(self.handle, ctypes.byref(c), nxt, ctypes.byref(lam.c),
                                       ctypes.c_void_p(grad3.data_ptr()), _stream_ptr(stream)))
        lam._pull()
        return lam

    def observables(self, st: DeviceState, stream=None) -> dict:
        out = (ctypes.c_double * 5)()
        rc = lib().drpf_observables(self.handle, ctypes.byref(st.c), out, 5, _stream_ptr(stream))
        if rc not in (DRPF_OK, DRPF_ENONFINITE):
            _check(rc)
        d = dict(zip(OBSERVABLES, list(out)))
        d["finite"] = rc == DRPF_OK
        return d

    def helmholtz_solve(self, rhs, which="fine", bc="neumann", coeff=1.0, shift=0.0, out=None,
                        wall=None, stream=None):
        """drpf_helmholtz_solve; ``wall`` (optional device tensor of two x-y layers, bottom then
        top) carries the inhomogeneous wall data of the boundary kind."""
        import torch
        x = torch.empty_like(rhs) if out is None else out
        wp = ctypes.c_void_p(wall.data_ptr()) if wall is not None else None
        _check(lib().drpf_helmholtz_solve(self.handle, 0 if which == "fine" else 1, BCS[bc],
                                          float(coeff), float(shift), ctypes.c_void_p(rhs.data_ptr()),
                                          wp, ctypes.c_void_p(x.data_ptr()), _stream_ptr(stream)))
        return x

    def helmholtz_solve_static(self, rhs, which="fine", bc="neumann", coeff=1.0, shift=0.0, out=None,
                               wall=None, stream=None):
        """drpf_helmholtz_solve_static: the same solve with the library's static scratch."""
        import torch
        x = torch.empty_like(rhs) if out is None else out
        wp = ctypes.c_void_p(wall.data_ptr()) if wall is not None else None
        _check(lib().drpf_helmholtz_solve_static(self.handle, 0 if which == "fine" else 1, BCS[bc],
                                                 float(coeff), float(shift), ctypes.c_void_p(rhs.data_ptr()),
                                                 wp, ctypes.c_void_p(x.data_ptr()), _stream_ptr(stream)))
        return x

    def prolong(self, u, v, w, stream=None):
        import torch
        uf = torch.empty(self.fine_shape, dtype=self.torch_dtype, device=self.device)
        vf = torch.empty_like(uf)
        wf = torch.empty_like(uf)
        _check(lib().drpf_prolong(self.handle, *(ctypes.c_void_p(a.data_ptr()) for a in (u, v, w, uf, vf, wf)),
                                  _stream_ptr(stream)))
        return uf, vf, wf

    def restrict(self, fine, location="center", stream=None):
        import torch
        loc = LOCATIONS[location]
        nz = self.coarse_shape[0] + (1 if loc in (3, 5, 6) else 0)
        out = torch.empty((nz,) + self.coarse_shape[1:], dtype=self.torch_dtype, device=self.device)
        _check(lib().drpf_restrict(self.handle, ctypes.c_void_p(fine.data_ptr()),
                                   ctypes.c_void_p(out.data_ptr()), loc, _stream_ptr(stream)))
        return out

    def profile_begin(self, max_launches: int, stream=None):
        _check(lib().drpf_profile_begin(self.handle, int(max_launches), _stream_ptr(stream)))

    def profile_end(self) -> dict:
        """{kernel name: (total ms, launches)} from the HIP events since profile_begin."""
        n = NKERNELS
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int * n)()
        _check(lib().drpf_profile_end(self.handle, ms, cnt, n))
        return {lib().drpf_kernel_name(k).decode(): (ms[k], cnt[k]) for k in range(n)}

    def debug_field(self, idx: int):
        """Copy of an internal coarse array (see drpf_debug_field) as a numpy array."""
        import torch
        ptr = ctypes.c_void_p()
        n = ctypes.c_size_t()
        _check(lib().drpf_debug_field(self.handle, int(idx), ctypes.byref(ptr), ctypes.byref(n)))
        esz = 8 if self.params.precision == 64 else 4
        b0 = ptr.value - self.workspace.data_ptr()
        raw = self.workspace[b0:b0 + int(n.value) * esz].clone().view(self.torch_dtype)
        nz = int(n.value) // (self.coarse_shape[1] * self.coarse_shape[2])
        return raw.reshape((nz,) + self.coarse_shape[1:]).double().cpu().numpy()
