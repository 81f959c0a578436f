"""ctypes binding of libvcsgc.so (the C ABI of include/vcsgc.h).

Argument marshalling only: every step of the sweep, the EAM evaluation and the
MD runs in the library's HIP kernels.  PyTorch supplies device memory and the
HIP stream.  There is no fallback: if the library is missing or no GPU is
present, constructing a context raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvcsgc.so")

STATUS = {0: "OK", -1: "INVALID_ARG", -2: "BOX_TOO_SMALL", -3: "OUT_OF_MEMORY", -4: "DEVICE",
          -5: "STATE", -6: "NO_SURROGATE", -7: "BARRIER_TIMEOUT", -8: "OVERFLOW"}


class VcsgcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"vcsgc error {code} ({STATUS.get(code, '?')}): {msg}")
        self.code = code


class EamFS(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("rc", "c0", "c1", "eps_aa", "eps_ab", "eps_bb", "t_a",
                                          "t_b", "a_a", "a_b", "mass_a", "mass_b")]


class EamTableC(C.Structure):
    _fields_ = [("nr", C.c_int32), ("nrho", C.c_int32), ("dr", C.c_double),
                ("drho", C.c_double), ("rc", C.c_double), ("f", C.c_void_p * 2),
                ("phi", C.c_void_p * 3), ("F", C.c_void_p * 2)]


class System(C.Structure):
    _fields_ = [("n_atoms", C.c_int64), ("box", C.c_double * 3),
                ("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p),
                ("vx", C.c_void_p), ("vy", C.c_void_p), ("vz", C.c_void_p),
                ("fx", C.c_void_p), ("fy", C.c_void_p), ("fz", C.c_void_p),
                ("species", C.c_void_p), ("pot", EamFS), ("skin", C.c_double),
                ("r_dep", C.c_double), ("flags", C.c_uint32),
                ("table", C.POINTER(EamTableC)), ("grow_edge", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("trials", C.c_int64), ("local_accepts", C.c_int64), ("stages", C.c_int64),
                ("stage_accepts", C.c_int64), ("flips", C.c_int64), ("near_ties", C.c_int64),
                ("n_final", C.c_int64), ("sum_n", C.c_double), ("sum_n2", C.c_double),
                ("stage1_pass", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TrainCfg(C.Structure):
    _fields_ = [("epochs", C.c_int64), ("batch", C.c_int64), ("lr", C.c_double),
                ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double),
                ("seed", C.c_uint64)]


class TrainReport(C.Structure):
    _fields_ = [("loss_first", C.c_double), ("loss_last", C.c_double), ("steps", C.c_int64)]


FLAG_DESCRIPTOR = 1
FLAG_COLOURS27 = 2
SURROGATE_MODES = {"off": 0, "mlp": 1, "perfect": 2, "zero": 3}
N_PARAMS = 4929


class State(C.Structure):
    _fields_ = [("sweeps_done", C.c_uint64), ("n_b", C.c_int64), ("seed", C.c_uint64),
                ("rho_dev", C.c_void_p)]


class Info(C.Structure):
    _fields_ = [("n_cells", C.c_int32 * 3), ("stages_per_sweep", C.c_int64), ("kmax", C.c_int32),
                ("mc_kmax_used", C.c_int32), ("mc_pairs", C.c_int64), ("md_pairs", C.c_int64),
                ("md_rebuilds", C.c_int64)]


KT_NAMES = ["trial", "commit", "density", "forces", "kick_drift", "kick", "build", "energy",
            "persist", "stage"]
STRATEGIES = {"graph": 0, "persistent": 1, "stage": 2, "batch": 3}


class CgParams(C.Structure):
    _fields_ = [("max_iter", C.c_int64), ("max_eval", C.c_int64), ("etol", C.c_double),
                ("ftol", C.c_double), ("dmax", C.c_double)]


class CgResult(C.Structure):
    _fields_ = [("iterations", C.c_int64), ("evaluations", C.c_int64), ("energy", C.c_double),
                ("fnorm", C.c_double), ("reason", C.c_int32)]


class KTimes(C.Structure):
    _fields_ = [("total_ms", C.c_double * len(KT_NAMES)), ("count", C.c_int64 * len(KT_NAMES)),
                ("launches", C.c_int64 * len(KT_NAMES))]


_lib = None
_P = C.c_void_p


def lib():
    """Load libvcsgc.so (after torch, so that one HIP runtime serves both)."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (binds the process to torch's HIP runtime first)
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        st = C.c_int
        L.vcsgc_create.restype = st
        L.vcsgc_create.argtypes = [C.POINTER(System), _P, C.POINTER(_P)]
        L.vcsgc_destroy.restype = st
        L.vcsgc_destroy.argtypes = [_P]
        L.vcsgc_sweep.restype = st
        L.vcsgc_sweep.argtypes = [_P, C.c_double, C.c_double, C.c_double, C.c_double, C.c_int64,
                                  C.c_uint64, C.POINTER(Stats)]
        L.eam_energy_forces.restype = st
        L.eam_energy_forces.argtypes = [_P, C.POINTER(C.c_double), C.c_int]
        L.md_verlet_step.restype = st
        L.md_verlet_step.argtypes = [_P, C.c_double, C.c_int64]
        L.vcsgc_last_error.restype = C.c_char_p
        L.vcsgc_last_error.argtypes = [_P]
        L.vcsgc_set_log.restype = st
        L.vcsgc_set_log.argtypes = [_P, _P, C.c_int64, _P, C.c_int64]
        L.vcsgc_log_counts.restype = st
        L.vcsgc_log_counts.argtypes = [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.vcsgc_get_state.restype = st
        L.vcsgc_get_state.argtypes = [_P, C.POINTER(State)]
        L.vcsgc_set_state.restype = st
        L.vcsgc_set_state.argtypes = [_P, C.POINTER(State)]
        L.vcsgc_copy_rho.restype = st
        L.vcsgc_copy_rho.argtypes = [_P, _P]
        L.vcsgc_atom_energies.restype = st
        L.vcsgc_atom_energies.argtypes = [_P, _P]
        L.vcsgc_get_info.restype = st
        L.vcsgc_get_info.argtypes = [_P, C.POINTER(Info)]
        L.vcsgc_kernel_timing.restype = st
        L.vcsgc_kernel_timing.argtypes = [_P, C.c_uint32]
        L.vcsgc_set_thermostat.restype = st
        L.vcsgc_set_thermostat.argtypes = [_P, C.c_double, C.c_double, C.c_double, C.c_double]
        L.vcsgc_get_thermostat.restype = st
        L.vcsgc_get_thermostat.argtypes = [_P, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.vcsgc_set_wait_limit.restype = st
        L.vcsgc_set_wait_limit.argtypes = [_P, C.c_uint32]
        L.vcsgc_set_local_steps.restype = st
        L.vcsgc_set_local_steps.argtypes = [_P, C.c_int32]
        L.vcsgc_kernel_timing_sampled.restype = st
        L.vcsgc_kernel_timing_sampled.argtypes = [_P, C.c_uint32, C.c_int32]
        L.vcsgc_get_kernel_timing.restype = st
        L.vcsgc_get_kernel_timing.argtypes = [_P, C.POINTER(KTimes)]
        L.vcsgc_create_batch.restype = st
        L.vcsgc_create_batch.argtypes = [C.POINTER(System), C.c_int32, _P, _P, _P, C.POINTER(_P)]
        L.vcsgc_sweep_batch.restype = st
        L.vcsgc_sweep_batch.argtypes = [_P, _P, _P, _P, _P, C.c_int64, C.c_uint64, _P]
        L.vcsgc_set_tuning.restype = st
        L.vcsgc_set_tuning.argtypes = [_P, C.c_int32, C.c_int32]
        L.vcsgc_get_tuning.restype = st
        L.vcsgc_get_tuning.argtypes = [_P, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                       C.POINTER(C.c_int32)]
        L.vcsgc_mlp_create.restype = st
        L.vcsgc_mlp_create.argtypes = [C.c_uint64, _P, C.POINTER(_P)]
        L.vcsgc_mlp_destroy.restype = st
        L.vcsgc_mlp_destroy.argtypes = [_P]
        L.vcsgc_mlp_set_params.restype = st
        L.vcsgc_mlp_set_params.argtypes = [_P, _P, _P, _P, C.c_float, C.c_float]
        L.vcsgc_mlp_get_params.restype = st
        L.vcsgc_mlp_get_params.argtypes = [_P, _P, _P, _P, C.POINTER(C.c_float),
                                           C.POINTER(C.c_float)]
        L.vcsgc_mlp_fit_normalization.restype = st
        L.vcsgc_mlp_fit_normalization.argtypes = [_P, _P, _P, C.c_int64]
        L.vcsgc_mlp_train.restype = st
        L.vcsgc_mlp_train.argtypes = [_P, _P, _P, C.c_int64, C.POINTER(TrainCfg),
                                      C.POINTER(TrainReport)]
        L.vcsgc_mlp_forward.restype = st
        L.vcsgc_mlp_forward.argtypes = [_P, _P, C.c_int64, _P]
        L.vcsgc_mlp_grad.restype = st
        L.vcsgc_mlp_grad.argtypes = [_P, _P, _P, C.c_int64, _P, C.POINTER(C.c_double)]
        L.vcsgc_mlp_grad_noalloc.restype = st
        L.vcsgc_mlp_grad_noalloc.argtypes = [_P, _P, _P, C.c_int64, _P, _P]
        L.vcsgc_set_sample_log.restype = st
        L.vcsgc_set_sample_log.argtypes = [_P, _P, _P, C.c_int64, C.c_int64]
        L.vcsgc_sample_count.restype = st
        L.vcsgc_sample_count.argtypes = [_P, C.POINTER(C.c_int64)]
        L.vcsgc_set_surrogate.restype = st
        L.vcsgc_set_surrogate.argtypes = [_P, _P, C.c_int32]
        L.vcsgc_set_surrogate_log.restype = st
        L.vcsgc_set_surrogate_log.argtypes = [_P, _P, C.c_int64]
        L.vcsgc_descriptors.restype = st
        L.vcsgc_descriptors.argtypes = [_P, _P, C.c_int64, C.c_int32, _P]
        L.vcsgc_selftest_sqrt.restype = st
        L.vcsgc_selftest_sqrt.argtypes = [_P, _P, C.c_int64, _P]
        L.vcsgc_selftest_md_math.restype = st
        L.vcsgc_selftest_md_math.argtypes = [_P, _P, _P, _P, C.c_int64, _P]
        L.vcsgc_set_barostat.restype = st
        L.vcsgc_set_barostat.argtypes = [_P, C.c_double, C.c_double, C.c_double]
        L.vcsgc_get_barostat.restype = st
        L.vcsgc_get_barostat.argtypes = [_P, C.POINTER(C.c_double), _P, C.POINTER(C.c_double)]
        L.vcsgc_minimize.restype = st
        L.vcsgc_minimize.argtypes = [_P, C.POINTER(CgParams), C.POINTER(CgResult)]
        _lib = L
    return _lib


def _stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev(a, dtype, device):
    import torch
    if isinstance(a, torch.Tensor):
        t = a.to(device=device, dtype=dtype)
    else:
        t = torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=device)
    return t.contiguous()


def pot_struct(pot, mass_a=55.845, mass_b=63.546) -> EamFS:
    """The analytic parameters, or for a tabulated potential (an object with
    rc, dr, drho and tables f, phi, F) only its cutoff and the masses."""
    if hasattr(pot, "phi"):
        return EamFS(float(pot.rc), *([0.0] * 9), mass_a, mass_b)
    return EamFS(*pot.as_tuple(), mass_a, mass_b)


def table_struct(pot):
    """(EamTableC, the host arrays it points to) for a tabulated potential,
    or (None, None).  The arrays must outlive the create call."""
    if not hasattr(pot, "phi"):
        return None, None
    keep = [np.ascontiguousarray(a, dtype=np.float64) for a in
            (pot.f[0], pot.f[1], pot.phi[0], pot.phi[1], pot.phi[2], pot.F[0], pot.F[1])]
    t = EamTableC()
    t.nr, t.nrho = int(keep[0].size), int(keep[5].size)
    t.dr, t.drho, t.rc = float(pot.dr), float(pot.drho), float(pot.rc)
    for k in range(2):
        t.f[k] = keep[k].ctypes.data
        t.F[k] = keep[5 + k].ctypes.data
    for k in range(3):
        t.phi[k] = keep[2 + k].ctypes.data
    return t, keep


def selftest_sqrt(x):
    """Device FP64 sqrt of a CUDA float64 tensor (diagnostic)."""
    import torch
    out = torch.empty_like(x)
    rc = lib().vcsgc_selftest_sqrt(_P(x.data_ptr()), _P(out.data_ptr()), x.numel(),
                                   _stream_handle())
    if rc:
        raise VcsgcError(rc, "selftest_sqrt")
    torch.cuda.synchronize()
    return out


def selftest_md_math(a, b):
    """(sqrt(a), a / b) as the MD passes compute them, for CUDA float64
    tensors a, b of one shape (diagnostic)."""
    import torch
    sq, q = torch.empty_like(a), torch.empty_like(a)
    rc = lib().vcsgc_selftest_md_math(_P(a.data_ptr()), _P(b.data_ptr()), _P(sq.data_ptr()),
                                      _P(q.data_ptr()), a.numel(), _stream_handle())
    if rc:
        raise VcsgcError(rc, "selftest_md_math")
    torch.cuda.synchronize()
    return sq, q


class VCSGC:
    """One system on the GPU.  Arrays are torch CUDA tensors owned by this
    object (copied from numpy inputs) and borrowed by the library context."""

    def __init__(self, x, y, z, box, species, pot, vx=None, vy=None, vz=None, forces=False,
                 skin=0.3, r_dep=0.0, mass_a=55.845, mass_b=63.546, device="cuda", stream=None,
                 descriptor=False, colours=8, grow_edge=0.0):
        import torch
        L = lib()
        self.device = torch.device(device)
        f64 = torch.float64
        self.x, self.y, self.z = (_dev(a, f64, self.device) for a in (x, y, z))
        self.species = _dev(species, torch.uint8, self.device)
        self.n = self.x.numel()
        self.box = np.asarray(box, dtype=np.float64)
        self.pot = pot
        self.vx = self.vy = self.vz = None
        if vx is not None:
            self.vx, self.vy, self.vz = (_dev(a, f64, self.device) for a in (vx, vy, vz))
        self.fx = self.fy = self.fz = None
        if forces or vx is not None:
            self.fx, self.fy, self.fz = (torch.zeros(self.n, dtype=f64, device=self.device)
                                         for _ in range(3))
        self.stream = stream
        sysd = System()
        sysd.n_atoms = self.n
        sysd.box = (C.c_double * 3)(*self.box.tolist())
        ptr = lambda t: None if t is None else t.data_ptr()  # noqa: E731
        sysd.x, sysd.y, sysd.z = ptr(self.x), ptr(self.y), ptr(self.z)
        sysd.vx, sysd.vy, sysd.vz = ptr(self.vx), ptr(self.vy), ptr(self.vz)
        sysd.fx, sysd.fy, sysd.fz = ptr(self.fx), ptr(self.fy), ptr(self.fz)
        sysd.species = ptr(self.species)
        sysd.pot = pot_struct(pot, mass_a, mass_b)
        tab, tab_keep = table_struct(pot)
        if tab is not None:
            sysd.table = C.pointer(tab)
        sysd.skin = float(skin)
        sysd.r_dep = float(r_dep)
        if colours not in (8, 27):
            raise ValueError("colours must be 8 or 27")
        sysd.flags = (FLAG_DESCRIPTOR if descriptor else 0) | (FLAG_COLOURS27 if colours == 27 else 0)
        sysd.grow_edge = float(grow_edge)
        self._sys = sysd
        h = _P()
        rc = L.vcsgc_create(C.byref(sysd), _stream_handle(stream), C.byref(h))
        if rc:
            raise VcsgcError(rc, L.vcsgc_last_error(None).decode())
        self._h = h
        self._logs = None

    # -- lifecycle ---------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            lib().vcsgc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc:
            msg = lib().vcsgc_last_error(self._h)
            raise VcsgcError(rc, f"{what}: {msg.decode() if msg else ''}")

    # -- calls --------------------------------------------------------------
    def sweep(self, dmu0, kappa, cbar, T, n_sweeps, seed, stats=True):
        s = Stats()
        self._check(lib().vcsgc_sweep(self._h, float(dmu0), float(kappa), float(cbar), float(T),
                                      int(n_sweeps), int(seed), C.byref(s) if stats else None),
                    "sweep")
        return s.as_dict() if stats else None

    def energy(self, forces=False):
        e = C.c_double()
        self._check(lib().eam_energy_forces(self._h, C.byref(e), int(bool(forces))), "energy")
        return e.value

    def compute_forces(self):
        self._check(lib().eam_energy_forces(self._h, None, 1), "forces")

    def md(self, dt, n_steps):
        self._check(lib().md_verlet_step(self._h, float(dt), int(n_steps)), "md")

    def set_barostat(self, p_ext, tau_p, pe=0.0):
        """Nose-Hoover barostat (p_ext in eV/A^3, tau_p in fs; 0: off) for
        later md() calls; needs the thermostat."""
        self._check(lib().vcsgc_set_barostat(self._h, float(p_ext), float(tau_p), float(pe)),
                    "set_barostat")

    def barostat(self):
        """(pe, box, virial) after the last NPT call."""
        pe, vir = C.c_double(), C.c_double()
        box = np.zeros(3)
        self._check(lib().vcsgc_get_barostat(self._h, C.byref(pe), box.ctypes.data_as(C.c_void_p),
                                             C.byref(vir)), "barostat")
        return pe.value, box, vir.value

    def minimize(self, max_iter=1000, max_eval=100000, etol=0.0, ftol=1e-6, dmax=0.1):
        """Conjugate-gradient relaxation of the positions (vcsgc_minimize);
        returns dict(iterations, evaluations, energy, fnorm, reason)."""
        p = CgParams(int(max_iter), int(max_eval), float(etol), float(ftol), float(dmax))
        r = CgResult()
        self._check(lib().vcsgc_minimize(self._h, C.byref(p), C.byref(r)), "minimize")
        return dict(iterations=r.iterations, evaluations=r.evaluations, energy=r.energy,
                    fnorm=r.fnorm, reason=r.reason)

    def set_thermostat(self, T, tau, xi=0.0, eta=0.0):
        """Nose-Hoover NVT for later md() calls (T = 0: NVE)."""
        self._check(lib().vcsgc_set_thermostat(self._h, float(T), float(tau), float(xi),
                                               float(eta)), "set_thermostat")

    def thermostat(self):
        """(xi, eta) of the thermostat."""
        xi, eta = C.c_double(), C.c_double()
        self._check(lib().vcsgc_get_thermostat(self._h, C.byref(xi), C.byref(eta)), "thermostat")
        return xi.value, eta.value

    def enable_log(self, trial_cap, stage_cap):
        import torch
        t = torch.zeros((max(trial_cap, 1), 8), dtype=torch.float64, device=self.device)
        s = torch.zeros((max(stage_cap, 1), 8), dtype=torch.float64, device=self.device)
        self._logs = (t, s, trial_cap, stage_cap)
        self._check(lib().vcsgc_set_log(self._h, _P(t.data_ptr()), int(trial_cap),
                                        _P(s.data_ptr()), int(stage_cap)), "set_log")

    def disable_log(self):
        self._check(lib().vcsgc_set_log(self._h, None, 0, None, 0), "set_log")
        self._logs = None

    def logs(self):
        """(trial log, stage log) as numpy arrays, rows sorted by (w, s, cell)."""
        import torch
        nt, ns = C.c_int64(), C.c_int64()
        self._check(lib().vcsgc_log_counts(self._h, C.byref(nt), C.byref(ns)), "log_counts")
        t, s, tc, sc = self._logs
        self._logs_n_trials = nt.value
        torch.cuda.synchronize()
        tl = t[:min(nt.value, tc)].cpu().numpy()
        sl = s[:min(ns.value, sc)].cpu().numpy()
        if tl.size:
            tl = tl[np.lexsort((tl[:, 2], tl[:, 1], tl[:, 0]))]
        if sl.size:
            sl = sl[np.lexsort((sl[:, 1], sl[:, 0]))]
        return tl, sl, nt.value, ns.value

    def get_state(self, with_rho=False):
        """Checkpoint: sweep counter, n_B, seed of the last call and, with
        with_rho, a device copy of the density cache."""
        import torch
        st = State()
        rho = None
        if with_rho:
            rho = torch.empty(self.n, dtype=torch.float64, device=self.device)
            st.rho_dev = rho.data_ptr()
        self._check(lib().vcsgc_get_state(self._h, C.byref(st)), "get_state")
        out = {"sweeps_done": st.sweeps_done, "n_b": st.n_b, "seed": st.seed}
        if with_rho:
            out["rho"] = rho
        return out

    def set_state(self, sweeps_done, seed=0, rho=None):
        """Resume: counter and seed; rho (a device tensor of N doubles) replaces
        the density cache."""
        st = State(int(sweeps_done), 0, int(seed), None if rho is None else rho.data_ptr())
        self._check(lib().vcsgc_set_state(self._h, C.byref(st)), "set_state")

    def rho(self):
        import torch
        out = torch.empty(self.n, dtype=torch.float64, device=self.device)
        self._check(lib().vcsgc_copy_rho(self._h, _P(out.data_ptr())), "copy_rho")
        torch.cuda.synchronize()
        return out

    def atom_energies(self):
        import torch
        out = torch.empty(self.n, dtype=torch.float64, device=self.device)
        self._check(lib().vcsgc_atom_energies(self._h, _P(out.data_ptr())), "atom_energies")
        torch.cuda.synchronize()
        return out

    def kernel_timing(self, names, every=1):
        """Time the launches of the named kernel classes with HIP events (resets);
        with every > 1 only one launch in `every` of each class is timed."""
        mask = 0
        for nm in names:
            mask |= 1 << KT_NAMES.index(nm)
        self._check(lib().vcsgc_kernel_timing_sampled(self._h, mask, int(every)),
                    "kernel_timing")

    def kernel_times(self):
        """{class: (total_ms, timed launches, all launches)} since kernel_timing()."""
        k = KTimes()
        self._check(lib().vcsgc_get_kernel_timing(self._h, C.byref(k)), "get_kernel_timing")
        return {nm: (k.total_ms[i], k.count[i], k.launches[i]) for i, nm in enumerate(KT_NAMES)
                if k.count[i]}

    def set_tuning(self, strategy="graph", trials_per_group=1):
        self._check(lib().vcsgc_set_tuning(self._h, STRATEGIES[strategy], int(trials_per_group)),
                    "set_tuning")

    def set_wait_limit(self, polls):
        """Polls before a persistent-sweep barrier wait is abandoned."""
        self._check(lib().vcsgc_set_wait_limit(self._h, int(polls)), "set_wait_limit")

    def set_local_steps(self, k):
        """Trials per active cell per stage (local chains; 1 = the plain scheme)."""
        self._check(lib().vcsgc_set_local_steps(self._h, int(k)), "set_local_steps")

    def tuning(self):
        a, b, g = C.c_int32(), C.c_int32(), C.c_int32()
        self._check(lib().vcsgc_get_tuning(self._h, C.byref(a), C.byref(b), C.byref(g)),
                    "get_tuning")
        inv = {v: k for k, v in STRATEGIES.items()}
        return {"strategy": inv[a.value], "trials_per_group": b.value, "workgroups": g.value}

    # -- surrogate ----------------------------------------------------------
    def set_surrogate(self, mode="off", mlp=None):
        self._mlp_ref = mlp
        self._check(lib().vcsgc_set_surrogate(self._h, None if mlp is None else mlp._h,
                                              SURROGATE_MODES[mode]), "set_surrogate")

    def enable_surrogate_log(self, cap):
        import torch
        self._dalog = torch.zeros((max(cap, 1), 5), dtype=torch.float64, device=self.device)
        self._dacap = cap
        self._check(lib().vcsgc_set_surrogate_log(self._h, _P(self._dalog.data_ptr()), int(cap)),
                    "set_surrogate_log")

    def surrogate_log(self):
        """(w, s, cell, dE_f, dE_r) rows sorted by (w, s, cell); call after logs()."""
        import torch
        torch.cuda.synchronize()
        n = min(int(self._logs_n_trials), self._dacap)
        a = self._dalog[:n].cpu().numpy()
        return a[np.lexsort((a[:, 2], a[:, 1], a[:, 0]))] if n else a

    def enable_sample_log(self, cap, stride):
        import torch
        self._smp_desc = torch.zeros((max(cap, 1), 10), dtype=torch.float64, device=self.device)
        self._smp_de = torch.zeros(max(cap, 1), dtype=torch.float64, device=self.device)
        self._smp_cap = cap
        self._check(lib().vcsgc_set_sample_log(self._h, _P(self._smp_desc.data_ptr()),
                                               _P(self._smp_de.data_ptr()), int(cap), int(stride)),
                    "set_sample_log")

    def disable_sample_log(self):
        self._check(lib().vcsgc_set_sample_log(self._h, None, None, 0, 1), "set_sample_log")

    def samples(self):
        """(descriptors [n][10], dE [n]) recorded so far, as device tensors."""
        n = C.c_int64()
        self._check(lib().vcsgc_sample_count(self._h, C.byref(n)), "sample_count")
        k = min(n.value, self._smp_cap)
        return self._smp_desc[:k], self._smp_de[:k]

    def descriptors(self, sites, flip=False):
        import torch
        s = torch.as_tensor(np.asarray(sites, dtype=np.int32), device=self.device)
        out = torch.zeros((s.numel(), 10), dtype=torch.float64, device=self.device)
        self._check(lib().vcsgc_descriptors(self._h, _P(s.data_ptr()), s.numel(), int(bool(flip)),
                                            _P(out.data_ptr())), "descriptors")
        torch.cuda.synchronize()
        return out.cpu().numpy()

    def info(self):
        i = Info()
        self._check(lib().vcsgc_get_info(self._h, C.byref(i)), "info")
        return {"n_cells": list(i.n_cells), "stages_per_sweep": i.stages_per_sweep,
                "kmax": i.kmax, "mc_kmax_used": i.mc_kmax_used, "mc_pairs": i.mc_pairs,
                "md_pairs": i.md_pairs, "md_rebuilds": i.md_rebuilds}


class VCSGCBatch(VCSGC):
    """Independent replicas in one context (MC only).  reps: list of dicts with
    x, y, z, box, species (numpy); arrays are concatenated on the device."""

    def __init__(self, reps, pot, r_dep=0.0, mass_a=55.845, mass_b=63.546, device="cuda",
                 stream=None, colours=8):
        import torch
        L = lib()
        self.device = torch.device(device)
        f64 = torch.float64
        cat = lambda k, dt: torch.as_tensor(np.concatenate([np.asarray(r[k]) for r in reps]),  # noqa: E731
                                            dtype=dt, device=self.device).contiguous()
        self.x, self.y, self.z = cat("x", f64), cat("y", f64), cat("z", f64)
        self.species = cat("species", torch.uint8)
        self.n = self.x.numel()
        self.n_rep = len(reps)
        self.rep_atoms = np.array([np.asarray(r["x"]).size for r in reps], dtype=np.int64)
        self.offsets = np.concatenate([[0], np.cumsum(self.rep_atoms)])
        self.rep_box = np.ascontiguousarray(np.stack([np.asarray(r["box"], dtype=np.float64)
                                                      for r in reps]))
        self.box = self.rep_box[0]
        self.pot = pot
        self.vx = self.vy = self.vz = self.fx = self.fy = self.fz = None
        sysd = System()
        sysd.n_atoms = self.n
        sysd.box = (C.c_double * 3)(*self.box.tolist())
        sysd.x, sysd.y, sysd.z = self.x.data_ptr(), self.y.data_ptr(), self.z.data_ptr()
        sysd.species = self.species.data_ptr()
        sysd.pot = pot_struct(pot, mass_a, mass_b)
        tab, tab_keep = table_struct(pot)
        if tab is not None:
            sysd.table = C.pointer(tab)
        sysd.skin = 0.3
        sysd.r_dep = float(r_dep)
        if colours not in (8, 27):
            raise ValueError("colours must be 8 or 27")
        sysd.flags = FLAG_COLOURS27 if colours == 27 else 0
        self._sys = sysd
        self.stream = stream
        h = _P()
        rc = L.vcsgc_create_batch(C.byref(sysd), self.n_rep,
                                  self.rep_atoms.ctypes.data_as(_P),
                                  self.rep_box.ctypes.data_as(_P), _stream_handle(stream),
                                  C.byref(h))
        if rc:
            raise VcsgcError(rc, L.vcsgc_last_error(None).decode())
        self._h = h
        self._logs = None

    def sweep_batch(self, dmu0, kappa, cbar, T, n_sweeps, seed, stats=True):
        arr = lambda v: np.ascontiguousarray(np.broadcast_to(np.asarray(v, dtype=np.float64),  # noqa: E731
                                                             (self.n_rep,)))
        d, k, c, t = arr(dmu0), arr(kappa), arr(cbar), arr(T)
        out = (Stats * self.n_rep)() if stats else None
        self._check(lib().vcsgc_sweep_batch(self._h, d.ctypes.data_as(_P), k.ctypes.data_as(_P),
                                            c.ctypes.data_as(_P), t.ctypes.data_as(_P),
                                            int(n_sweeps), int(seed), out), "sweep_batch")
        return [s.as_dict() for s in out] if stats else None

    def replica_species(self, r):
        a, b = self.offsets[r], self.offsets[r + 1]
        return self.species[a:b].cpu().numpy()

    def replica_rho(self, r):
        rho = self.rho().cpu().numpy()
        return rho[self.offsets[r]:self.offsets[r + 1]]


class Mlp:
    """Surrogate network handle (device parameters, training, inference)."""

    def __init__(self, seed=0, stream=None):
        h = _P()
        rc = lib().vcsgc_mlp_create(int(seed), _stream_handle(stream), C.byref(h))
        if rc:
            raise VcsgcError(rc, "mlp_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().vcsgc_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc:
            raise VcsgcError(rc, what)

    def set_params(self, flat, mu, sd, out_mu, out_sd):
        f = lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.float32))  # noqa: E731
        p, m, s = f(flat), f(mu), f(sd)
        self._check(lib().vcsgc_mlp_set_params(self._h, p.ctypes.data_as(_P), m.ctypes.data_as(_P),
                                               s.ctypes.data_as(_P), float(out_mu), float(out_sd)),
                    "set_params")

    def get_params(self):
        p = np.zeros(N_PARAMS, dtype=np.float32)
        mu = np.zeros(10, dtype=np.float32)
        sd = np.zeros(10, dtype=np.float32)
        om, osd = C.c_float(), C.c_float()
        self._check(lib().vcsgc_mlp_get_params(self._h, p.ctypes.data_as(_P), mu.ctypes.data_as(_P),
                                               sd.ctypes.data_as(_P), C.byref(om), C.byref(osd)),
                    "get_params")
        return p, mu, sd, om.value, osd.value

    def fit_normalization(self, desc, dE):
        self._check(lib().vcsgc_mlp_fit_normalization(self._h, _P(desc.data_ptr()),
                                                      _P(dE.data_ptr()), desc.shape[0]),
                    "fit_normalization")

    def train(self, desc, dE, epochs=10, batch=4096, lr=1e-3, seed=0):
        cfg = TrainCfg(int(epochs), int(batch), float(lr), 0.9, 0.999, 1e-8, int(seed))
        rep = TrainReport()
        self._check(lib().vcsgc_mlp_train(self._h, _P(desc.data_ptr()), _P(dE.data_ptr()),
                                          desc.shape[0], C.byref(cfg), C.byref(rep)), "train")
        return {"loss_first": rep.loss_first, "loss_last": rep.loss_last, "steps": rep.steps}

    def forward(self, desc):
        import torch
        out = torch.zeros(desc.shape[0], dtype=torch.float64, device=desc.device)
        self._check(lib().vcsgc_mlp_forward(self._h, _P(desc.data_ptr()), desc.shape[0],
                                            _P(out.data_ptr())), "forward")
        torch.cuda.synchronize()
        return out

    def grad(self, desc, dE):
        g = np.zeros(N_PARAMS, dtype=np.float32)
        loss = C.c_double()
        self._check(lib().vcsgc_mlp_grad(self._h, _P(desc.data_ptr()), _P(dE.data_ptr()),
                                         desc.shape[0], g.ctypes.data_as(_P), C.byref(loss)),
                    "grad")
        return loss.value, g

    def grad_noalloc(self, desc, dE, grad_out, loss_out):
        """vcsgc_mlp_grad_noalloc: gradient and mean loss of n <= 4096 samples
        into caller device tensors (float32[4929], float64[1]); asynchronous."""
        self._check(lib().vcsgc_mlp_grad_noalloc(self._h, _P(desc.data_ptr()),
                                                 _P(dE.data_ptr()), desc.shape[0],
                                                 _P(grad_out.data_ptr()),
                                                 _P(loss_out.data_ptr())), "grad_noalloc")
