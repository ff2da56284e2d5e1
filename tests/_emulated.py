"""The library's HIP sources built as host code against the CPU stand-in for
HIP in tests/emu (every GPU thread a fiber, barriers and wavefront
exchanges emulated, device memory as exact-size heap blocks under
AddressSanitizer), plus writers of the case files tests/emu/driver.cpp
reads.  Test infrastructure: it checks the kernels' indexing, barriers and
results on the CPU; it shares no arithmetic with the oracle."""
import ctypes
import os
import re
import shutil
import struct
import subprocess
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2307_13483_amd", "csrc")
EMU = os.path.join(ROOT, "tests", "emu")
CXX = "/opt/rocm/llvm/bin/clang++"
FLAGS = ["-std=c++20", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address", "-pthread",
         "-Wno-unused-function", "-Wno-unknown-attributes"]
# the dynamic LDS array of the kernels becomes the launch's heap block
_DYN_LDS = re.compile(r"^extern __shared__ __align__\(16\) char vdc_tile_lds\[\];$", re.M)


def available():
    return os.path.exists(CXX)


def build(outdir, jobs=8):
    """Compile every library source and the driver; returns the driver path."""
    src = os.path.join(outdir, "src")
    obj = os.path.join(outdir, "obj")
    os.makedirs(src, exist_ok=True)
    os.makedirs(obj, exist_ok=True)
    for f in os.listdir(CSRC):
        if f.endswith((".h", ".hip")):
            shutil.copy(os.path.join(CSRC, f), src)
    found = 0
    for f in os.listdir(src):
        path = os.path.join(src, f)
        text, n = _DYN_LDS.subn("#define vdc_tile_lds emu_dyn_lds", open(path).read())
        if n:
            open(path, "w").write(text)
            found += n
    if found == 0:
        raise RuntimeError("no dynamic LDS declaration found in the sources")
    inc = ["-I", os.path.join(EMU, "include"), "-I", os.path.join(ROOT, "include"), "-I", src]
    units = [os.path.join(src, f) for f in sorted(os.listdir(src)) if f.endswith(".hip")]
    units += [os.path.join(EMU, "emu_fiber.cpp"), os.path.join(EMU, "driver.cpp")]

    def compile_one(u):
        o = os.path.join(obj, os.path.basename(u) + ".o")
        r = subprocess.run([CXX, *FLAGS, *inc, "-x", "c++", "-c", u, "-o", o],
                           stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        if r.returncode:
            raise RuntimeError(f"{u}:\n{r.stdout[-4000:]}")
        return o

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_one, units))
    exe = os.path.join(outdir, "vdc_emu")
    r = subprocess.run([CXX, "-fsanitize=address", "-pthread", *objs, "-o", exe],
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode:
        raise RuntimeError(r.stdout[-4000:])
    return exe


def run(exe, args, timeout=900, **env):
    """Run the driver; returns (exit code, output).  AddressSanitizer reports
    (and aborts with) any access outside an allocation."""
    e = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", EMU_THREADS="4")
    e.update({k: str(v) for k, v in env.items()})
    r = subprocess.run([exe, *args], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                       timeout=timeout, env=e)
    return r.returncode, r.stdout


def job_lines(out):
    """(status, iters, outer, rel_res, retried) of every job line."""
    rows = []
    for line in out.splitlines():
        m = re.match(r"job \d+ status (\d+) iters (\d+) outer (\d+) rel_res (\S+) retried (\d+)", line)
        if m:
            rows.append((int(m[1]), int(m[2]), int(m[3]), float(m[4]), int(m[5])))
    return rows


def _model2d_desc(vdc, p, Ng, Nu):
    d = vdc.ModelDesc()
    d.omega_g, d.omega_u = p["omega_g"], p["omega_u"]
    d.kappa1, d.kappa2, d.lam = p["kappa1"], p["kappa2"], p["lam"]
    d.lam1, d.lam2 = p["lam1"], p["lam2"]
    d.E1, d.gap = p["E1"], p["gap"]
    for s, st in enumerate(("1", "2")):
        for m, mu in enumerate(("e", "o")):
            d.A[s][m] = p["A" + st + mu]
            d.B[s][m] = p["B" + st + mu]
    d.l[0], d.l[1] = int(p["l_e"]), int(p["l_o"])
    d.Ng, d.Nu = int(Ng), int(Nu)
    d.hilbert_nodes, d.hilbert_xmax = int(p.get("K", 4096)), float(p.get("X", 40.0))
    return d


def write_solve_case(path, models, jobs, finals, opts):
    """models: [(params, Ng, Nu)]; jobs: (eps_i, (v_g, v_u), mu, model)."""
    from paper_2307_13483_amd import vdc
    with open(path, "wb") as f:
        f.write(struct.pack("<i", len(models)))
        for (p, Ng, Nu) in models:
            f.write(bytes(_model2d_desc(vdc, p, Ng, Nu)))
        f.write(struct.pack("<i", len(jobs)))
        for (e, v, mu, k) in jobs:
            f.write(bytes(vdc.Job(float(e), int(v[0]), int(v[1]), int(mu), int(k))))
        f.write(struct.pack("<i", len(finals)))
        for fv in finals:
            f.write(struct.pack("<ii", int(fv[0]), int(fv[1])))
        f.write(bytes(opts.c()))


def write_co2_desc(path, params, sizes):
    from paper_2307_13483_amd import vdc
    d = vdc.Co2Desc()
    for k in vdc.CO2_PARAMS:
        setattr(d, k, float(params[k]))
    for c, cn in enumerate(("sigma", "pi")):
        for w, wn in enumerate(("s", "p")):
            d.A[c][w] = float(params["A_%s_%s" % (cn, wn)])
            d.B[c][w] = float(params["B_%s_%s" % (cn, wn)])
    d.Ns, d.Nx, d.Ny, d.Na = (int(sizes[k]) for k in ("s", "x", "y", "a"))
    d.hilbert_nodes = int(params.get("K", 4096))
    d.hilbert_xmax = float(params.get("X", 40.0))
    open(path, "wb").write(bytes(d))


def write_terms_case(path, desc, jobs, finals, opts):
    """desc as paper_2307_13483_amd.inputs builds it; jobs (eps_i, v, mu)."""
    from paper_2307_13483_amd import vdc
    D, M, P = len(desc["e_state"]), len(desc["nbasis"]), len(desc["l"])
    with open(path, "wb") as f:
        f.write(struct.pack("<iii", D, M, P))
        f.write(struct.pack("<%dd" % M, *desc["omega"]))
        f.write(struct.pack("<%di" % M, *desc["nbasis"]))
        f.write(struct.pack("<%dd" % D, *desc["e_state"]))
        for key in ("uterms", "vterms"):
            f.write(struct.pack("<i", len(desc[key])))
            for (d, e, c, pw) in desc[key]:
                t = vdc.Term()
                t.d, t.e, t.coeff = int(d), int(e), float(c)
                for q, pq in enumerate(pw):
                    t.pow[q] = int(pq)
                f.write(bytes(t))
        for dd in range(D):
            for mu in range(P):
                A, B = desc["width"].get((dd, mu), (0.0, 1.0))
                f.write(bytes(vdc.Width(float(A), float(B), int(desc["l"][mu]))))
        f.write(struct.pack("<id", int(desc.get("K", 4096)), float(desc.get("X", 40.0))))
        f.write(struct.pack("<i", len(jobs)))
        mj = vdc._mjobs(jobs)
        f.write(bytes(mj)[:len(jobs) * ctypes.sizeof(vdc.MJob)])
        f.write(struct.pack("<i", len(finals)))
        for fv in finals:
            row = [0] * vdc.MAX_MODES
            for q, vq in enumerate(fv):
                row[q] = int(vq)
            f.write(struct.pack("<%di" % vdc.MAX_MODES, *row))
        f.write(bytes(opts.c()))


def write_co2_solve_case(path, jobs, finals, opts):
    """jobs: (eps_i, (n_s, n_x, n_y, n_a), mu_i); finals: 4-tuples."""
    from paper_2307_13483_amd import vdc
    with open(path, "wb") as f:
        f.write(struct.pack("<i", len(jobs)))
        for (e, v, mu) in jobs:
            j = vdc.Co2Job()
            j.eps_i = float(e)
            for q in range(4):
                j.v[q] = int(v[q])
            j.mu_i = int(mu)
            f.write(bytes(j))
        f.write(struct.pack("<i", len(finals)))
        for fv in finals:
            f.write(struct.pack("<4i", *[int(c) for c in fv]))
        f.write(bytes(opts.c()))
