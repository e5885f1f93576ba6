"""Algorithm 1 (Sec. 2.3): hard-kill topology optimisation on voxels, driven through the library's C ABI.

Per iteration: boundary of the material voxels -> 4 triangles per face (geometry.cantilever_problem),
BEM solve (bem_solve), stress at the filled voxel centres (bem_stress, eq. stress_1), topological
derivative (kfmm_topological_derivative, eq. deriv), removal of the voxels below
D_min + C (D_max - D_min), post-processing, volume ratio alpha and compliance Psi.

Readings where the paper is silent: the first and last voxel layers along the beam (clamped and loaded
ends) are protected from removal; post-processing keeps the voxels face-connected to both protected
layers (a floating piece would make the elastic problem singular).

DeviceOptimiser runs the same iteration with every step in the library (boundary extraction, targets, the
adaptive two-scale sampling of Sec. 5, removal and post-processing), the design kept on the device.

The warm-start study (`warm_start_study`) re-solves the systems of a fixed sequence with three starting
points -- zero, the previous solution mapped onto the new surface, and the learned network (with the
residual guard) -- and reports GMRES iterations and times.
"""
import time

import numpy as np
import torch

from workloads import geometry as geo


def _dev(x, dt=torch.float64):
    return torch.tensor(np.ascontiguousarray(x), dtype=dt, device="cuda")


def postprocess(M):
    """Keep the voxels face-connected to both end layers (x = 0 and x = nx - 1)."""
    from scipy import ndimage
    lab, n = ndimage.label(M)
    if n == 0:
        return M
    lo = set(np.unique(lab[0][lab[0] > 0]))
    hi = set(np.unique(lab[-1][lab[-1] > 0]))
    keep = sorted(lo & hi)
    return np.isin(lab, keep) & M


def voxel_centres(M, h):
    idx = np.argwhere(M)
    return (idx + 0.5) * h, idx


class Problem:
    """Surface problem of a voxel set on the device."""

    def __init__(self, M, h, load):
        p = geo.cantilever_problem(M, h, load)
        self.host = p
        self.T = p["tri"].shape[0]
        self.dev = dict(tri=_dev(p["tri"]), bc_type=_dev(p["bc_type"], torch.int8), bc_val=_dev(p["bc_val"]))

    def args(self):
        return (self.dev["tri"], self.dev["bc_type"], self.dev["bc_val"])


class Optimiser:
    def __init__(self, M0, h=1.0, load=(0.0, 0.0, -1.0), C=0.02, G=1.0, nu=0.3, tol=1e-8, restart=200, p=8,
                 leaf_max=128, precision=0, max_iter=5000, precond=0, m2l_tol=0.0):
        from paper_1612_04082_amd import kfmm
        self.kfmm = kfmm
        self.M0 = np.asarray(M0, bool)
        self.h, self.load, self.C = h, load, C
        self.G, self.nu = G, nu
        self.K = kfmm.moduli(G, nu)
        self.E = 2 * G * (1 + nu)
        self.solve_kw = dict(K=self.K, G=G, tol=tol, restart=restart, p=p, leaf_max=leaf_max, precision=precision,
                             max_iter=max_iter, precond=precond, m2l_tol=m2l_tol)
        self.fmm_kw = dict(K=self.K, G=G, p=p, leaf_max=leaf_max, precision=precision, m2l_tol=m2l_tol)

    def solve(self, prob, x0=None, x0_alt=None, **over):
        kw = dict(self.solve_kw)
        kw.update(over)
        return self.kfmm.bem_solve(*prob.args(), x0=x0, x0_alt=x0_alt, allow_noconv=True, **kw)

    def evaluate(self, M, prob, u, t):
        """Stress, topological derivative and energy density at the filled voxel centres."""
        trg, idx = voxel_centres(M, self.h)
        sig = self.kfmm.bem_stress(*prob.args(), u, t, _dev(trg), **self.fmm_kw)
        td = self.kfmm.topological_derivative(sig, K=self.K, G=self.G).cpu().numpy()
        s = sig.cpu().numpy()
        ss = (s[:, :3] ** 2).sum(1) + 2 * (s[:, 3:] ** 2).sum(1)
        tr = s[:, :3].sum(1)
        energy = 0.5 * ((1 + self.nu) * ss - self.nu * tr * tr) / self.E
        return idx, td, energy

    def remove(self, M, idx, td):
        lo, hi = td.min(), td.max()
        kill = td < lo + self.C * (hi - lo)
        kill &= (idx[:, 0] > 0) & (idx[:, 0] < M.shape[0] - 1)  # protected end layers
        M2 = M.copy()
        M2[tuple(idx[kill].T)] = False
        return postprocess(M2)

    def run(self, n_iter, alpha_c=0.0, callback=None):
        M = self.M0.copy()
        hist = []
        for k in range(n_iter):
            prob = Problem(M, self.h, self.load)
            x, u, t, st = self.solve(prob)
            idx, td, energy = self.evaluate(M, prob, u, t)
            alpha = M.sum() / self.M0.sum()
            psi = energy.sum() * self.h ** 3
            hist.append(dict(iter=k + 1, alpha=float(alpha), psi=float(psi), T=prob.T, gmres=st["iters"],
                             rel_res=st["rel_res"]))
            if callback:
                callback(k, M, prob, x, u, t, st)
            if alpha < alpha_c:
                break
            M_next = self.remove(M, idx, td)
            if not M_next.any():  # the rule would disconnect the supports: stop with the last design
                break
            M = M_next
        return M, hist


class DeviceOptimiser(Optimiser):
    """Algorithm 1 with every step in the library: boundary extraction (alg1_surface), the solve, stress at
    the voxel centres (alg1_centres, or the adaptive two-round sampling with blocks of `block` voxels:
    alg1_coarse_blocks, alg1_refine, alg1_expand), the topological derivative and the removal rule with
    post-processing (alg1_update).  The design stays on the device; the host only sequences the calls."""

    def __init__(self, M0, block=0, **kw):
        super().__init__(M0, **kw)
        self.block = int(block)

    def step_fields(self, vox, prob, u, t):
        """TD per filled voxel (linear order), the number of stress points evaluated, and the compliance
        (uniform sampling only; None with the adaptive sampling)."""
        k = self.kfmm
        args = (prob["tri"], prob["bc_type"], prob["bc_val"])
        if self.block <= 1:
            trg = k.alg1_centres(vox, self.h)
            sig = k.bem_stress(*args, u, t, trg, **self.fmm_kw)
            td = k.topological_derivative(sig, K=self.K, G=self.G)
            return td, int(trg.shape[0]), k.alg1_energy(sig, self.K, self.G) * self.h ** 3
        b = self.block
        tc = k.alg1_coarse_blocks(vox, self.h, b)
        td_c = (k.topological_derivative(k.bem_stress(*args, u, t, tc, **self.fmm_kw), K=self.K, G=self.G)
                if tc.shape[0] else torch.empty(0, dtype=torch.float64, device=vox.device))
        tf, _ = k.alg1_refine(vox, self.h, b, td_c, self.C)
        td_f = (k.topological_derivative(k.bem_stress(*args, u, t, tf, **self.fmm_kw), K=self.K, G=self.G)
                if tf.shape[0] else torch.empty(0, dtype=torch.float64, device=vox.device))
        td = k.alg1_expand(vox, self.h, b, td_c, self.C, td_f)
        return td, int(tc.shape[0] + tf.shape[0]), None

    def run(self, n_iter, alpha_c=0.0, callback=None):
        k = self.kfmm
        vox = torch.tensor(np.ascontiguousarray(self.M0), dtype=torch.uint8, device="cuda")
        n0 = int(self.M0.sum())
        hist = []
        for it in range(n_iter):
            prob = k.alg1_surface(vox, self.h, self.load)
            x, u, t, st = k.bem_solve(prob["tri"], prob["bc_type"], prob["bc_val"], x0=None, allow_noconv=True,
                                      **self.solve_kw)
            td, n_eval, psi = self.step_fields(vox, prob, u, t)
            n_filled = int(td.shape[0])
            alpha = n_filled / n0
            hist.append(dict(iter=it + 1, alpha=float(alpha), psi=psi, T=int(prob["tri"].shape[0]), gmres=st["iters"],
                             rel_res=st["rel_res"], stress_points=n_eval))
            if callback:
                callback(it, vox, prob, x, u, t, st)
            if alpha < alpha_c:
                break
            nxt, kept = k.alg1_update(vox, self.h, td, self.C)
            if kept == 0:  # the rule would disconnect the supports: stop with the last design
                break
            vox = nxt
        return vox.cpu().numpy().astype(bool), hist


def warm_start_study(M0, n_iter=20, train_from=2, measure_from=11, h=1.0, C=0.02, tol_seq=1e-8, tol=1e-6,
                     epochs=200, lr=1e-3, seed=0, log=print, **kw):
    """Drive Algorithm 1 with tight solves; re-solve the measured systems from three starts.

    Returns a list of per-iteration records (iterations and seconds for x0 = 0, previous, network)."""
    from paper_1612_04082_amd import kfmm
    opt = Optimiser(M0, h=h, C=C, tol=tol_seq, **kw)
    net = kfmm.WarmStartNet(seed=seed)
    rec = []
    state = {}

    def sync():
        torch.cuda.synchronize()

    def cb(k, M, prob, x, u, t, st):
        r = dict(iter=k + 1, T=prob.T, seq_iters=st["iters"])
        if "prev" in state:
            pv = state["prev"]
            sync()
            t0 = time.time()
            feat, xm, scale = kfmm.ws_features(pv["prob"].dev, pv["u"], pv["t"], prob.dev)
            sync()
            t_feat = time.time() - t0
            if k + 1 >= measure_from:
                for mode in ("zero", "prev", "net"):
                    sync()
                    t0 = time.time()
                    if mode == "zero":
                        _, _, _, s2 = opt.solve(prob, tol=tol)
                        extra = 0.0
                    elif mode == "prev":
                        _, _, _, s2 = opt.solve(prob, x0=xm, tol=tol)
                        extra = t_feat
                    else:
                        t1 = time.time()
                        x0 = net.predict(feat, xm, scale)
                        sync()
                        extra = t_feat + (time.time() - t1)
                        _, _, _, s2 = opt.solve(prob, x0=x0, x0_alt=xm, tol=tol)
                    sync()
                    r[mode] = dict(iters=s2["iters"], seconds=time.time() - t0 + extra, rel_res0=s2["rel_res0"],
                                   rel_res_start=s2["rel_res_start"] if mode != "zero" else 1.0,
                                   converged=s2["converged"], used_alt=s2.get("used_alt", 0),
                                   used_zero=s2.get("used_zero", 0))
            if k + 1 >= train_from:
                sync()
                t0 = time.time()
                r["train_loss"] = net.train(feat, xm, x, scale, epochs=epochs, lr=lr)
                sync()
                r["train_seconds"] = time.time() - t0
        state["prev"] = dict(prob=prob, u=u.clone(), t=t.clone())
        rec.append(r)
        log(r)

    _, hist = opt.run(n_iter, callback=cb)
    for r, hh in zip(rec, hist):
        r.update(alpha=hh["alpha"], psi=hh["psi"])
    net.close()
    return rec


# ---------------------------------------------------------------------------------- periodic cell (Sec. 4.3)

def hashin_shtrikman_bulk(K, G, f_void):
    """Hashin-Shtrikman upper bound of the bulk modulus of a porous isotropic material (void fraction f)."""
    return K + f_void / (-1.0 / K + 3.0 * (1.0 - f_void) / (3.0 * K + 4.0 * G))


class PeriodicCell:
    """The metamaterial cell of Sec. 4.3 on the device: a cubic voxel cell repeated over the lattice, the
    superposition formulation (the fluctuation field carries -s^h n on the void/material faces, the total
    stress is s^h plus it), hydrostatic s^h for the bulk modulus.

    single_iteration(alpha_c): the paper's single-iteration solution -- solve once on the initial design,
    topological derivative (eq. deriv) of the total stress at every filled voxel centre, keep the largest
    values at the volume fraction alpha_c (alg1_cell_surface, bem_solve and bem_stress on the periodic cell,
    alg1_centres, alg1_cell_td, alg1_cell_update).
    bulk_modulus(vox): effective bulk modulus of a design: <sigma> = C : [eps_h (1 - f) + (1/V) sum_e A_e
    sym(u_e (x) n_e)] with the solution u on the faces (n_e out of the material, eps_h the matrix strain of
    s^h; a rigid translation of u drops out on closed surfaces), K_eff = <sigma>_kk / (3 tr eps_h)."""

    def __init__(self, n, h=None, K=None, G=1.0, p=8, leaf_max=64, tol=1e-6, restart=100, max_iter=400,
                 m2l_tol=0.0, near_levels=0):
        from paper_1612_04082_amd import kfmm
        self.kfmm = kfmm
        self.n = int(n)
        self.h = 1.0 / n if h is None else float(h)
        self.L = self.n * self.h
        self.G = G
        self.K = kfmm.moduli(G, 0.3) if K is None else K
        self.cell = (0.0, 0.0, 0.0, self.L)
        self.sig_h = (1.0, 1.0, 1.0, 0.0, 0.0, 0.0)
        self.fmm_kw = dict(K=self.K, G=G, p=p, leaf_max=leaf_max, precision=kfmm.FP64, cell=self.cell,
                           m2l_tol=m2l_tol)
        self.solve_kw = dict(self.fmm_kw, tol=tol, restart=restart, max_iter=max_iter, near_levels=near_levels)

    def _sync_time(self, t0):
        torch.cuda.synchronize()
        return time.time() - t0

    def solve(self, vox):
        k = self.kfmm
        t0 = time.time()
        prob = k.alg1_cell_surface(vox, self.h, self.sig_h)
        t_surf = self._sync_time(t0)
        t0 = time.time()
        x, u, t, st = k.bem_solve(prob["tri"], prob["bc_type"], prob["bc_val"], allow_noconv=True, **self.solve_kw)
        t_solve = self._sync_time(t0)
        return prob, u, t, dict(T=int(prob["tri"].shape[0]), gmres=st["iters"], rel_res=st["rel_res"],
                                converged=bool(st["converged"]), t_surface_s=t_surf, t_solve_s=t_solve)

    def bulk_modulus(self, vox, prob=None, u=None):
        if prob is None:
            prob, u, _, rec = self.solve(vox)
        else:
            rec = {}
        tri = prob["tri"].cpu().numpy()
        uu = u.cpu().numpy()
        cr = np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0])
        area_n = 0.5 * cr  # A_e n_e
        f = 1.0 - float((vox != 0).float().mean().item())
        V = self.L ** 3
        eps_h = np.eye(3) / (3.0 * self.K)  # s^h = I
        E = eps_h * (1.0 - f) + np.einsum("ei,ej->ij", uu, area_n) / V
        E = 0.5 * (E + E.T)
        K_eff = self.K * np.trace(E) / np.trace(eps_h)  # <sigma>_kk = 3 K tr E
        rec.update(void_fraction=f, K_eff=float(K_eff), K_hs=float(hashin_shtrikman_bulk(self.K, self.G, f)))
        return rec

    def single_iteration(self, M0, alpha_c):
        k = self.kfmm
        vox = _dev(M0, torch.uint8)
        prob, u, t, rec = self.solve(vox)
        rec.update(self.bulk_modulus(vox, prob, u))
        t0 = time.time()
        pts = k.alg1_centres(vox, self.h)
        sig = k.bem_stress(prob["tri"], prob["bc_type"], prob["bc_val"], u, t, pts, **self.fmm_kw)
        rec["t_stress_s"] = self._sync_time(t0)
        rec["stress_points"] = int(pts.shape[0])
        t0 = time.time()
        td = k.alg1_cell_td(sig, self.sig_h, K=self.K, G=self.G)
        new, kept = k.alg1_cell_update(vox, self.h, td, alpha_c)
        rec["t_update_s"] = self._sync_time(t0)
        rec["kept"] = kept
        return new, rec
