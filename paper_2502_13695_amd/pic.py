"""ctypes binding of libpic.so (include/pic.h).

Argument marshalling only: every step of the method runs in the HIP kernels
behind the C ABI.  The library must be built (``python -m
paper_2502_13695_amd.build``); loading fails loudly otherwise.  PyTorch, when
present with a GPU, provides the device allocator and the stream.
"""

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpic.so")
_LIB = None

PIC_OK = 0
STATUS = {0: "ok", -1: "invalid argument", -2: "device allocation failed", -3: "HIP runtime error",
          -4: "invalid state (latched error)", -5: "non-finite value",
          -6: "charged-particle capacity exceeded", -7: "ABI version mismatch"}
ABI_VERSION = 2
ENV = {"gauss": 0, "sin2": 1}
BC = {"outflow": 0, "periodic": 1}
DIAG_SCALARS, DIAG_FIELDS, DIAG_NE, DIAG_UE, DIAG_EVENTS, DIAG_PARTICLES, DIAG_PARAMS, DIAG_AMP, \
    DIAG_TIMERS, DIAG_SORT, DIAG_REGION, DIAG_IMAX, DIAG_TRACKS, DIAG_HEALTH, DIAG_POL = range(15)
SC = dict(step=0, time=1, n_neutral=2, n_e=3, n_pos=4, events=5, u_field=6, ke_e=7, ke_pos=8,
          e_gap=9, e_abs=10, gauss_max=11, rho_max=12, health=13, slots=14, tracks_dropped=15,
          gauss_l2=16, e_in=17, e_out=18)


class PicError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {STATUS.get(code, code)} ({code})")
        self.code = code


class Material(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("gap_eV", "n_index", "density_gcc", "molar_mass_gmol",
                                            "me_star", "mh_star", "pos_mass_kg", "lorentz_lambda_m",
                                            "eps_inf", "lorentz_gamma_s", "impact_rate_s", "kerr_n2_m2W")]


class Layer(C.Structure):
    _fields_ = [("material", C.c_int32), ("reserved", C.c_int32), ("lo_m", C.c_double),
                ("hi_m", C.c_double)]


class Laser(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("lambda_m", "fwhm_s", "peak_Wcm2", "fluence_Jcm2",
                                            "waist_m", "t_peak_s", "cep_rad")] + \
               [("envelope", C.c_int32), ("pol_axis", C.c_int32)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Config(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("abi_version", C.c_uint32), ("ndim", C.c_int32),
                ("transverse_bc", C.c_int32), ("n", C.c_int64 * 3), ("dx_m", C.c_double * 3),
                ("cfl", C.c_double), ("nsteps", C.c_int64), ("nmat", C.c_int32),
                ("nlayer", C.c_int32), ("mats", C.POINTER(Material)), ("layers", C.POINTER(Layer)),
                ("ppc", C.c_int32), ("shape_order", C.c_int32), ("T_K", C.c_double),
                ("keldysh_terms", C.c_int32), ("keldysh_tol_bits", C.c_int32), ("seed", C.c_uint64),
                ("laser", Laser), ("particle_capacity", C.c_int64), ("preionize_eV", C.c_double),
                ("collisions", C.c_int32), ("reserved2", C.c_int32), ("stream", C.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN),
                ("alloc_user", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("dt", C.c_double), ("Cd", C.c_double * 3), ("kmur", C.c_double * 3),
                ("ie", C.c_double * 8), ("nwin", C.c_int64), ("E0", C.c_double),
                ("t_peak", C.c_double), ("amp_cut", C.c_double * 8), ("amp_sat", C.c_double * 8),
                ("n_neutral", C.c_int64), ("capacity", C.c_int64), ("lor", (C.c_double * 3) * 8),
                ("chi3", C.c_double * 8)]


class Particle(C.Structure):
    _fields_ = [("cell", C.c_int32 * 3), ("kind", C.c_int32), ("off", C.c_float * 3),
                ("u", C.c_float * 3)]


PARTICLE_DTYPE = np.dtype([("cell", "<i4", 3), ("kind", "<i4"), ("off", "<f4", 3), ("u", "<f4", 3)])
assert PARTICLE_DTYPE.itemsize == C.sizeof(Particle)
# pic_track: a recorded position of a sampled particle
TRACK_DTYPE = np.dtype([("id", "<u4"), ("kind", "<i4"), ("step", "<i4"), ("cell", "<i4", 3),
                        ("off", "<f4", 3), ("reserved", "<i4")])
assert TRACK_DTYPE.itemsize == 40


class State(C.Structure):
    _fields_ = [("step", C.c_int64), ("E", C.POINTER(C.c_float) * 3), ("b", C.POINTER(C.c_float) * 3),
                ("n_particles", C.c_int64), ("particles", C.POINTER(Particle)),
                ("reset_window", C.c_int32), ("reserved", C.c_int32)]


SYMBOLS = ["pic_init", "pic_step", "pic_diag", "pic_set_state", "pic_footprint", "pic_canonical",
           "pic_keldysh_rate", "pic_table_probe", "pic_table_bound_probe", "pic_table_probe_device",
           "pic_batch_create",
           "pic_batch_step", "pic_batch_add", "pic_batch_remove", "pic_batch_destroy", "pic_batch_set_graph",
           "pic_batch_graph_replays",
           "pic_set_timing", "pic_autotune", "pic_autotune_steps", "pic_set_resort", "pic_set_far_tiles",
           "pic_set_imax", "pic_spectrum_counts", "pic_spectrum_counts_noalloc", "pic_set_tracks",
           "pic_snapshot", "pic_restore",
           "pic_destroy", "pic_status_str"]


class Spectrum(C.Structure):
    _fields_ = [("nedges", C.c_int32), ("edges_eV", C.POINTER(C.c_double)),
                ("x_lo_cell", C.c_int64), ("x_hi_cell", C.c_int64)]


def lib():
    """Load libpic.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_2502_13695_amd.build")
        # torch ships its own HIP runtime; load it first so that libpic.so binds
        # to the same runtime (one device context, torch-allocated memory valid)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        sig = {
            "pic_init": ([C.POINTER(Config), C.POINTER(vp)], C.c_int),
            "pic_step": ([vp, i64], C.c_int),
            "pic_diag": ([vp, C.c_int, vp, C.c_size_t, C.POINTER(C.c_size_t)], C.c_int),
            "pic_set_state": ([vp, C.POINTER(State)], C.c_int),
            "pic_footprint": ([C.POINTER(Config), C.POINTER(C.c_size_t)], C.c_int),
            "pic_canonical": ([C.POINTER(Config), C.POINTER(Params)], C.c_int),
            "pic_keldysh_rate": ([C.POINTER(Material), C.c_double, i32, C.POINTER(C.c_double), i64,
                                  C.POINTER(C.c_double)], C.c_int),
            "pic_table_probe": ([C.POINTER(Config), i32, C.POINTER(C.c_float), i64,
                                 C.POINTER(C.c_float)], C.c_int),
            "pic_table_bound_probe": ([C.POINTER(Config), i32, C.POINTER(C.c_float), i64,
                                       C.POINTER(C.c_float)], C.c_int),
            "pic_table_probe_device": ([vp, i32, C.POINTER(C.c_float), i64, C.POINTER(C.c_float)],
                                       C.c_int),
            "pic_batch_create": ([C.POINTER(vp), i32, C.POINTER(vp)], C.c_int),
            "pic_batch_step": ([vp, i64], C.c_int),
            "pic_batch_add": ([vp, vp], C.c_int),
            "pic_batch_remove": ([vp, vp], C.c_int),
            "pic_batch_destroy": ([vp], None),
            "pic_set_timing": ([vp, i32], C.c_int),
            "pic_autotune": ([vp, i32], C.c_int),
            "pic_autotune_steps": ([vp, i32], C.c_int),
            "pic_set_resort": ([vp, i32], C.c_int),
            "pic_set_far_tiles": ([vp, i32], C.c_int),
            "pic_set_imax": ([vp, i32], C.c_int),
            "pic_set_tracks": ([vp, C.c_uint32, i32, i64], C.c_int),
            "pic_snapshot": ([vp, vp, C.c_size_t, C.POINTER(C.c_size_t)], C.c_int),
            "pic_restore": ([vp, vp, C.c_size_t], C.c_int),
            "pic_spectrum_counts": ([vp, C.POINTER(Spectrum), C.POINTER(C.c_uint64), C.c_size_t], C.c_int),
            "pic_spectrum_counts_noalloc": ([vp, C.POINTER(Spectrum), C.POINTER(C.c_uint64), C.c_size_t],
                                            C.c_int),
            "pic_batch_set_graph": ([vp, i32], C.c_int),
            "pic_batch_graph_replays": ([vp], C.c_int64),
            "pic_destroy": ([vp], None),
            "pic_status_str": ([C.c_int], C.c_char_p),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _LIB = L
    return _LIB


def _check(code, what):
    if code != PIC_OK:
        raise PicError(code, what)


def make_config(cfg, stream=None, alloc=None, free=None):
    """Marshal a workload dictionary into a pic_config.  Returns (Config, keepalive)."""
    mats = (Material * max(1, len(cfg["materials"])))()
    for i, m in enumerate(cfg["materials"]):
        for k in ("gap_eV", "n_index", "density_gcc", "molar_mass_gmol", "me_star", "mh_star"):
            setattr(mats[i], k, float(m[k]))
        mats[i].pos_mass_kg = float(m.get("pos_mass_kg", 0.0))
        mats[i].lorentz_lambda_m = float(m.get("lorentz_lambda_m", 0.0))
        mats[i].eps_inf = float(m.get("eps_inf", 1.0))
        mats[i].lorentz_gamma_s = float(m.get("lorentz_gamma_s", 0.0))
        mats[i].impact_rate_s = float(m.get("impact_rate_s", 0.0))
        mats[i].kerr_n2_m2W = float(m.get("kerr_n2_m2W", 0.0))
    layers = (Layer * max(1, len(cfg["layers"])))()
    for i, (m, lo, hi) in enumerate(cfg["layers"]):
        layers[i].material = int(m)
        layers[i].lo_m = float(lo)
        layers[i].hi_m = float(hi)
    c = Config()
    c.struct_size = C.sizeof(Config)
    c.abi_version = ABI_VERSION
    c.ndim = int(cfg["ndim"])
    c.transverse_bc = BC[cfg.get("transverse_bc", "outflow")]
    for d in range(c.ndim):
        c.n[d] = int(cfg["n"][d])
        c.dx_m[d] = float(cfg["dx"][d])
    c.cfl = float(cfg["cfl"])
    c.nsteps = int(cfg["nsteps"])
    c.nmat = len(cfg["materials"])
    c.nlayer = len(cfg["layers"])
    c.mats = mats
    c.layers = layers
    c.ppc = int(cfg["ppc"])
    c.shape_order = int(cfg.get("shape_order", 2))
    c.T_K = float(cfg.get("T_K", 300.0))
    c.keldysh_terms = int(cfg.get("keldysh_terms", 500))
    c.keldysh_tol_bits = int(cfg.get("keldysh_tol_bits", 0))
    c.seed = int(cfg["seed"])
    L = cfg["laser"]
    for k in ("lambda_m", "fwhm_s", "cep_rad", "waist_m", "t_peak_s"):
        setattr(c.laser, k, float(L.get(k, 0.0)))
    c.laser.peak_Wcm2 = float(L.get("peak_Wcm2", 0.0))
    c.laser.fluence_Jcm2 = float(L.get("fluence_Jcm2", 0.0))
    c.laser.envelope = ENV[L.get("envelope", "gauss")]
    c.laser.pol_axis = int(L.get("pol_axis", 1))
    c.particle_capacity = int(cfg.get("particle_capacity", 0))
    c.preionize_eV = float(cfg.get("preionize_eV", 0.0))
    c.collisions = int(bool(cfg.get("collisions", False)))
    c.stream = stream
    if alloc is not None:
        c.alloc = alloc
        c.free = free
    return c, (mats, layers, alloc, free)


def _torch_allocator():
    """Device allocator callbacks backed by torch's caching allocator."""
    import torch
    dev = torch.cuda.current_device()

    def _a(nbytes, user):
        try:
            return int(torch.cuda.caching_allocator_alloc(int(nbytes), dev))
        except Exception:
            return None

    def _f(ptr, user):
        torch.cuda.caching_allocator_delete(ptr)

    return ALLOC_FN(_a), FREE_FN(_f)


def domain_shape(ndim, n, periodic_t, which, comp):
    out = []
    for d in range(3):
        if d >= ndim:
            out.append(1)
            continue
        half = (d == comp) if which == "E" else (d != comp)
        out.append(n[d] if (half or (periodic_t and d > 0)) else n[d] + 1)
    return tuple(out)


class Context:
    """One run (pic_init .. pic_destroy)."""

    def __init__(self, cfg, use_torch=True):
        L = lib()
        self.cfg = cfg
        self._keep = []
        stream = None
        alloc = free = None
        if use_torch:
            try:
                import torch
                if torch.cuda.is_available():
                    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
                    alloc, free = _torch_allocator()
            except ImportError:
                pass
        c, keep = make_config(cfg, stream=stream, alloc=alloc, free=free)
        self._config = c
        self._keep.append(keep)
        h = C.c_void_p()
        _check(L.pic_init(C.byref(c), C.byref(h)), "pic_init")
        self.h = h
        self.ndim = int(cfg["ndim"])
        self.n = [int(cfg["n"][d]) if d < self.ndim else 1 for d in range(3)]
        self.periodic_t = cfg.get("transverse_bc", "outflow") == "periodic"
        self.nmat = len(cfg["materials"])

    # -------------------------------------------------------------- control
    def step(self, n=1):
        _check(lib().pic_step(self.h, int(n)), "pic_step")

    def set_timing(self, on):
        _check(lib().pic_set_timing(self.h, int(on)), "pic_set_timing")

    def autotune_steps(self, reps=8):
        """Time every field tile shape on the next reps x shapes steps of the run
        (identical results) and keep the fastest."""
        _check(lib().pic_autotune_steps(self.h, int(reps)), "pic_autotune_steps")

    def set_resort(self, period):
        """Tile-sort check period in steps (0 = never sort the charged particles)."""
        _check(lib().pic_set_resort(self.h, int(period)), "pic_set_resort")

    def autotune(self, reps=20):
        """Pick the fastest field-kernel tile shape (before the first step)."""
        _check(lib().pic_autotune(self.h, int(reps)), "pic_autotune")
        t = self.timers()
        return dict(chosen=int(t[23]), blocks=int(t[24]), ms=[float(x) for x in t[16:23]])

    def close(self):
        if getattr(self, "h", None):
            lib().pic_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------- diagnostics
    def _diag_bytes(self, kind):
        n = C.c_size_t()
        _check(lib().pic_diag(self.h, kind, None, 0, C.byref(n)), "pic_diag(size)")
        return n.value

    def _diag(self, kind, dtype):
        nb = self._diag_bytes(kind)
        buf = np.zeros(max(1, nb // np.dtype(dtype).itemsize), dtype=dtype)
        w = C.c_size_t()
        _check(lib().pic_diag(self.h, kind, buf.ctypes.data_as(C.c_void_p), buf.nbytes, C.byref(w)),
               "pic_diag")
        return buf[: w.value // np.dtype(dtype).itemsize]

    def scalars(self):
        v = self._diag(DIAG_SCALARS, np.float64)
        return {k: float(v[i]) for k, i in SC.items()}

    def health(self):
        """Device health word, latched status, device step index, slots in use."""
        v = self._diag(DIAG_HEALTH, np.float64)
        return dict(bits=int(v[0]), latched=int(v[1]), step=int(v[2]), slots=int(v[3]))

    def _split(self, flat, which_list):
        out = []
        o = 0
        for which, comp in which_list:
            shp = domain_shape(self.ndim, self.n, self.periodic_t, which, comp)
            cnt = shp[0] * shp[1] * shp[2]
            out.append(flat[o:o + cnt].reshape(shp[::-1]).transpose(2, 1, 0))
            o += cnt
        return out

    def fields(self):
        """(E, b): lists of 3 FP64 arrays indexed [i, j, k] on their own positions."""
        flat = self._diag(DIAG_FIELDS, np.float64)
        arrs = self._split(flat, [("E", 0), ("E", 1), ("E", 2), ("b", 0), ("b", 1), ("b", 2)])
        return arrs[:3], arrs[3:]

    def polarisation(self):
        """(Q, K) of the Lorentz media: lists of 3 FP64 arrays on the E positions."""
        flat = self._diag(DIAG_POL, np.float64)
        arrs = self._split(flat, [("E", 0), ("E", 1), ("E", 2), ("E", 0), ("E", 1), ("E", 2)])
        return arrs[:3], arrs[3:]

    def _node_grid(self, kind, dtype):
        flat = self._diag(kind, dtype)
        shp = domain_shape(self.ndim, self.n, self.periodic_t, "node", -1)
        shp = tuple(self.n[d] + (0 if (self.periodic_t and d > 0) else 1) if d < self.ndim else 1
                    for d in range(3))
        return flat.reshape(shp[::-1]).transpose(2, 1, 0)

    def ne_grid(self):
        return self._node_grid(DIAG_NE, np.float64)

    def ue_grid(self):
        return self._node_grid(DIAG_UE, np.float64)

    def amp(self):
        return self._node_grid(DIAG_AMP, np.float32)

    def set_imax(self, every):
        """Sample the node |E|^2 into its running maximum after every
        `every`-th step (0 = off); enabling clears the maximum."""
        _check(lib().pic_set_imax(self.h, int(every)), "pic_set_imax")

    def imax(self):
        """Maximum accumulated intensity: the largest node |E|^2 [V^2/m^2]."""
        return self._node_grid(DIAG_IMAX, np.float32)

    def snapshot(self):
        """The whole simulation state as bytes (pic_snapshot)."""
        w = C.c_size_t()
        _check(lib().pic_snapshot(self.h, None, 0, C.byref(w)), "pic_snapshot(size)")
        buf = np.empty(w.value, dtype=np.uint8)
        _check(lib().pic_snapshot(self.h, buf.ctypes.data_as(C.c_void_p), buf.nbytes, C.byref(w)), "pic_snapshot")
        return buf

    def restore(self, snap):
        """Load a snapshot of a context with the same configuration."""
        b = np.ascontiguousarray(snap, dtype=np.uint8)
        _check(lib().pic_restore(self.h, b.ctypes.data_as(C.c_void_p), b.nbytes), "pic_restore")

    def set_tracks(self, fraction, every, max_records=1 << 20):
        """Record the position of a sampled `fraction` of the particles (by
        Philox draw on their id) after every `every`-th step (0 = off)."""
        thr = int(min(max(float(fraction), 0.0), 1.0) * 2.0 ** 32)
        _check(lib().pic_set_tracks(self.h, min(thr, 2 ** 32 - 1), int(every), int(max_records)),
               "pic_set_tracks")

    def tracks(self):
        """Recorded positions (TRACK_DTYPE), sorted by (id, kind, step)."""
        nb = self._diag_bytes(DIAG_TRACKS)
        buf = np.zeros(nb // TRACK_DTYPE.itemsize, dtype=TRACK_DTYPE)
        w = C.c_size_t()
        if nb:
            _check(lib().pic_diag(self.h, DIAG_TRACKS, buf.ctypes.data_as(C.c_void_p), buf.nbytes,
                                  C.byref(w)), "pic_diag(tracks)")
        return buf

    def spectrum(self, edges_eV, x_lo_cell=0, x_hi_cell=0):
        """Macroparticle counts per kind (rows) by kinetic energy over the bin
        edges [eV]: below the first edge, each bin, at or above the last edge."""
        e = np.ascontiguousarray(edges_eV, dtype=np.float64)
        nk = 2 * self.nmat
        out = np.zeros((nk, len(e) + 1), dtype=np.uint64)
        sp = Spectrum(len(e), e.ctypes.data_as(C.POINTER(C.c_double)), int(x_lo_cell), int(x_hi_cell))
        _check(lib().pic_spectrum_counts(self.h, C.byref(sp), out.ctypes.data_as(C.POINTER(C.c_uint64)),
                                         out.size), "pic_spectrum_counts")
        return out

    def spectrum_noalloc(self, edges_eV, x_lo_cell=0, x_hi_cell=0):
        """The energy histogram through the library's fixed device staging (no
        device allocation; calls on one GPU must not overlap)."""
        e = np.ascontiguousarray(edges_eV, dtype=np.float64)
        nk = 2 * self.nmat
        out = np.zeros((nk, len(e) + 1), dtype=np.uint64)
        sp = Spectrum(len(e), e.ctypes.data_as(C.POINTER(C.c_double)), int(x_lo_cell), int(x_hi_cell))
        _check(lib().pic_spectrum_counts_noalloc(self.h, C.byref(sp),
                                                 out.ctypes.data_as(C.POINTER(C.c_uint64)), out.size),
               "pic_spectrum_counts_noalloc")
        return out

    def events(self):
        v = self._diag(DIAG_EVENTS, np.int64)
        return v.reshape(-1, 2)

    def particles(self):
        nb = self._diag_bytes(DIAG_PARTICLES)
        buf = np.zeros(nb // PARTICLE_DTYPE.itemsize, dtype=PARTICLE_DTYPE)
        w = C.c_size_t()
        if nb:
            _check(lib().pic_diag(self.h, DIAG_PARTICLES, buf.ctypes.data_as(C.c_void_p), buf.nbytes,
                                  C.byref(w)), "pic_diag(particles)")
        return buf

    def params(self):
        p = Params()
        w = C.c_size_t()
        _check(lib().pic_diag(self.h, DIAG_PARAMS, C.byref(p), C.sizeof(p), C.byref(w)), "pic_diag(params)")
        return p

    def timers(self):
        return self._diag(DIAG_TIMERS, np.float64)

    def set_far_tiles(self, on):
        """Field tiles far from every charged particle so far skip the current."""
        _check(lib().pic_set_far_tiles(self.h, int(on)), "pic_set_far_tiles")

    def region(self):
        """Charged region along x of the next step (cells lo..hi, with the
        amplitude window), the field tiles that read / skip the current, the
        field front (last x node of a tile that held a nonzero field) and the
        field tiles updated so far over all field launches."""
        v = self._diag(DIAG_REGION, np.float64)
        return dict(lo=int(v[0]), hi=int(v[1]), near_tiles=int(v[2]), far_tiles=int(v[3]),
                    front=int(v[4]), tiles_updated=int(v[5]))

    def sort_state(self):
        """Tile-sort state: sorted slots, chunks, drifter-steps since the sort, sorts done."""
        v = self._diag(DIAG_SORT, np.float64)
        return dict(sorted=int(v[0]), chunks=int(v[1]), drift=int(v[2]), sorts=int(v[3]))

    def set_state(self, step, E=None, b=None, particles=None, reset_window=True):
        """Overwrite fields ([i, j, k] arrays on their own positions), charged
        particles (PARTICLE_DTYPE records) and the step index."""
        S = State()
        S.step = int(step)
        keep = []
        for q in range(3):
            for arrs, name in ((E, "E"), (b, "b")):
                if arrs is None:
                    continue
                a = np.ascontiguousarray(np.asarray(arrs[q], dtype=np.float32).transpose(2, 1, 0)).ravel()
                keep.append(a)
                getattr(S, name)[q] = a.ctypes.data_as(C.POINTER(C.c_float))
        if particles is not None and len(particles):
            p = np.ascontiguousarray(particles, dtype=PARTICLE_DTYPE)
            keep.append(p)
            S.n_particles = len(p)
            S.particles = p.ctypes.data_as(C.POINTER(Particle))
        S.reset_window = int(bool(reset_window))
        _check(lib().pic_set_state(self.h, C.byref(S)), "pic_set_state")

    def table_probe_device(self, mat, A):
        A = np.ascontiguousarray(A, dtype=np.float32)
        P = np.zeros_like(A)
        _check(lib().pic_table_probe_device(self.h, int(mat), A.ctypes.data_as(C.POINTER(C.c_float)),
                                            len(A), P.ctypes.data_as(C.POINTER(C.c_float))),
               "pic_table_probe_device")
        return P


class Batch:
    """Independent instances advanced together, one launch per phase."""

    def __init__(self, contexts=()):
        arr = (C.c_void_p * max(1, len(contexts)))(*[c.h for c in contexts])
        h = C.c_void_p()
        _check(lib().pic_batch_create(arr, len(contexts), C.byref(h)), "pic_batch_create")
        self.h = h

    def step(self, n=1):
        _check(lib().pic_batch_step(self.h, int(n)), "pic_batch_step")

    def set_graph(self, on):
        """Replay sort periods of batch steps as a HIP graph (default) or step eagerly."""
        _check(lib().pic_batch_set_graph(self.h, int(on)), "pic_batch_set_graph")

    def graph_replays(self):
        return int(lib().pic_batch_graph_replays(self.h))

    def add(self, ctx):
        _check(lib().pic_batch_add(self.h, ctx.h), "pic_batch_add")

    def remove(self, ctx):
        _check(lib().pic_batch_remove(self.h, ctx.h), "pic_batch_remove")

    def close(self):
        if getattr(self, "h", None):
            lib().pic_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------ host-only calls
def canonical(cfg):
    c, keep = make_config(cfg)
    p = Params()
    _check(lib().pic_canonical(C.byref(c), C.byref(p)), "pic_canonical")
    return p


def footprint(cfg):
    c, keep = make_config(cfg)
    n = C.c_size_t()
    _check(lib().pic_footprint(C.byref(c), C.byref(n)), "pic_footprint")
    return n.value


def keldysh_rate(material, lam, A, terms=500):
    m = Material()
    for k in ("gap_eV", "n_index", "density_gcc", "molar_mass_gmol", "me_star", "mh_star"):
        setattr(m, k, float(material[k]))
    A = np.ascontiguousarray(A, dtype=np.float64)
    W = np.zeros_like(A)
    _check(lib().pic_keldysh_rate(C.byref(m), float(lam), int(terms),
                                  A.ctypes.data_as(C.POINTER(C.c_double)), len(A),
                                  W.ctypes.data_as(C.POINTER(C.c_double))), "pic_keldysh_rate")
    return W


def table_probe(cfg, mat, A, bound=False):
    """Host lookup of the FP32 rate table at amplitudes A; with bound=True the
    skip bound of the ionization step instead (pic_table_bound_probe)."""
    c, keep = make_config(cfg)
    A = np.ascontiguousarray(A, dtype=np.float32)
    P = np.zeros_like(A)
    fn = "pic_table_bound_probe" if bound else "pic_table_probe"
    _check(getattr(lib(), fn)(C.byref(c), int(mat), A.ctypes.data_as(C.POINTER(C.c_float)), len(A),
                              P.ctypes.data_as(C.POINTER(C.c_float))), fn)
    return P
