"""Float64 restatement of the CoG training phase and cascade for tiny images.

An independent, pure-Python model used to cross-check the binary32 oracle on
4x4 inputs: it computes the kernel weights from math.exp, keeps the KDE
masses as exact integers, and carries the mixture, running average and
confidence in float64.  Decisions can differ from the binary32 oracle only
at threshold ties; the tests flag those.
"""
import math

import numpy as np


def kde_weights64(h=8.0):
    den = 2.0 * h * h
    z = math.fsum(math.exp(-(e * e) / den) for e in range(-1024, 1025))
    W = np.zeros((16, 256), dtype=np.int64)
    for b in range(16):
        for v in range(256):
            s = math.fsum(math.exp(-((u - v) ** 2) / den) for u in range(16 * b, 16 * b + 16)) / z
            W[b, v] = int(round(65535.0 * s))
    return W


class Brute:
    def __init__(self, width, height, channels, K, prm):
        self.P = width * height
        self.C = channels
        self.K = K
        self.p = prm
        self.W = kde_weights64(prm["kde_h"])

    # -- mixture step -------------------------------------------------------
    def gmm(self, comp, x, ae):
        """comp: list of [w, mu(list), var]; returns (label, m_post, margin)."""
        p, K = self.p, self.K
        cum, B = 0.0, K
        margin = float("inf")
        for b in range(K):
            cum += comp[b][0]
            margin = min(margin, abs(cum - p["T"]))
            if cum > p["T"]:
                B = b + 1
                break
        m = -1
        for k in range(K):
            w, mu, var = comp[k]
            if not w > 0:
                continue
            d2 = sum((x[c] - mu[c]) ** 2 for c in range(self.C))
            margin = min(margin, abs(d2 - p["lam"] ** 2 * var) / max(1.0, d2))
            if d2 <= p["lam"] ** 2 * var:
                m = k
                break
        lab = 0 if (m >= 0 and m < B) else 1
        om = 1.0 - ae
        for k in range(K):
            comp[k][0] *= om
        if m >= 0:
            comp[m][0] += ae
            rho = ae / comp[m][0]
            comp[m][1] = [(1 - rho) * comp[m][1][c] + rho * x[c] for c in range(self.C)]
            s = sum((x[c] - comp[m][1][c]) ** 2 for c in range(self.C))
            comp[m][2] = max(p["var_min"], (1 - rho) * comp[m][2] + rho * s)
        else:
            comp[K - 1] = [ae, list(x), p["var_init"]]
        S = sum(c[0] for c in comp)
        for k in range(K):
            comp[k][0] /= S
        order = list(range(K))
        # stable sort by w/sigma descending
        keyed = sorted(order, key=lambda k: -(comp[k][0] / math.sqrt(comp[k][2])))
        keys = [comp[k][0] / math.sqrt(comp[k][2]) for k in keyed]
        for k in range(K - 1):
            if keys[k] > 0:
                # equal sort keys are a tie: either order is a valid result
                margin = min(margin, (keys[k] - keys[k + 1]) / keys[k])
        new = [comp[k] for k in keyed]
        mp = keyed.index(m) if m >= 0 else -1
        comp[:] = new
        return lab, mp, margin

    # -- training -------------------------------------------------------------
    def train(self, frames):
        """frames: [N, P, C] ints."""
        p, C, K = self.p, self.C, self.K
        N = len(frames)
        self.N = N
        self.comp, self.rga, self.table, self.cnt = [], [], [], []
        self.label, self.prev = [], []
        for px in range(self.P):
            xs = [[float(frames[j][px][c]) for c in range(C)] for j in range(N)]
            comp = [[1.0, list(xs[0]), p["var_init"]]] + \
                   [[0.0, [0.0] * C, p["var_init"]] for _ in range(K - 1)]
            acc = [[0] * 16 for _ in range(C)]
            cnt = [0, 0, 0]
            lab = 0
            for j in range(N):
                for c in range(C):
                    v = int(xs[j][c])
                    for b in range(16):
                        acc[c][b] += int(self.W[b, v])
                if j >= 1:
                    dl = max(abs(xs[j][c] - xs[j - 1][c]) for c in range(C))
                    cnt[0 if dl < p["res_e1"] else (1 if dl < p["res_e2"] else 2)] += 1
                    lab, _, _ = self.gmm(comp, xs[j], p["alpha"])
            tab = []
            for c in range(C):
                amax = max(acc[c])
                tab.append([(255 * a + amax // 2) // amax for a in acc[c]])
            self.comp.append(comp)
            self.rga.append([list(comp[0][1]), comp[0][2]])
            self.table.append(tab)
            self.cnt.append(cnt)
            self.label.append(lab)
            self.prev.append(list(xs[-1]))
        self.sat = [0] * self.P
        self.frame = N

    # -- cascade ----------------------------------------------------------------
    def halted(self, blk):
        """Sampling: a block of 64 pixels whose pixels all have a saturated
        confidence is evaluated only when (frame + block) % period == 0."""
        p = self.p
        if not (p["stage_mask"] & 8) or (self.frame + blk) % p["samp_period"] == 0:
            return False
        pix = range(64 * blk, min(self.P, 64 * blk + 64))
        return all(self.sat[q] >= p["samp_window"] for q in pix)

    def step(self, frame):
        """frame: [P, C] ints.  Returns (mask list, stages list, margins list);
        stage -1 marks a pixel of a halted block."""
        p, C = self.p, self.C
        sm = p["stage_mask"]
        masks, stages, margins = [], [], []
        halted = [self.halted(b) for b in range((self.P + 63) // 64)]
        for px in range(self.P):
            if halted[px // 64]:
                masks.append(255 if self.label[px] else 0)
                stages.append(-1)
                margins.append(float("inf"))
                continue
            confident = False
            x = [float(frame[px][c]) for c in range(C)]
            xp = self.prev[px]
            mu_r, var_r = self.rga[px]
            margin = float("inf")
            dl = max(abs(x[c] - xp[c]) for c in range(C))
            if (sm & 1) and dl <= p["tau_fd"]:
                lab, st = self.label[px], 0
                confident = True
            else:
                dr2 = sum((x[c] - mu_r[c]) ** 2 for c in range(C))
                margin = min(margin, abs(dr2 - p["lambda_rga"] ** 2 * var_r) / max(1.0, dr2))
                if (sm & 2) and dr2 <= p["lambda_rga"] ** 2 * var_r:
                    lab, st = 0, 1
                    if sm & 8:
                        ls2 = p["samp_lambda"] ** 2 * var_r
                        confident = dr2 <= ls2
                        margin = min(margin, abs(dr2 - ls2) / max(1.0, dr2))
                    ar = p["alpha_rga"]
                    mu_r = [(1 - ar) * mu_r[c] + ar * x[c] for c in range(C)]
                    s = sum((x[c] - mu_r[c]) ** 2 for c in range(C))
                    var_r = max(p["var_min"], (1 - ar) * var_r + ar * s)
                    self.rga[px] = [mu_r, var_r]
                else:
                    conf = 0.0
                    st = 3
                    if sm & 4:
                        tb = self.table[px]
                        prod = 1
                        for c in range(C):
                            prod *= tb[c][int(x[c]) >> 4]
                        ph = prod / 255.0 ** C
                        a, b, g = (v / (self.N - 1) for v in self.cnt[px])
                        if ph < p["p_null"]:
                            a = 0.0
                        margin = min(margin, abs(ph - p["p_null"]))
                        dh = max(0.0, 1.0 - dl / p["res_e2"])
                        mh = max(0.0, 1.0 - dr2 / (p["lambda_m"] ** 2 * var_r))
                        conf = a * ph + b * dh + g * mh
                        margin = min(margin, abs(conf - p["conf_thr"]))
                        if conf >= p["conf_thr"]:
                            lab, st = 0, 2
                    if st == 3:
                        ae = p["alpha"] * (1.0 - p["kappa_alpha"] * conf)
                        lab, mp, mg = self.gmm(self.comp[px], x, ae)
                        margin = min(margin, mg)
                        if lab == 0:
                            self.rga[px] = [list(self.comp[px][mp][1]), self.comp[px][mp][2]]
            self.label[px] = lab
            self.prev[px] = x
            if sm & 8:
                self.sat[px] = min(self.sat[px] + 1, 65535) if confident else 0
            masks.append(255 if lab else 0)
            stages.append(st)
            margins.append(margin)
        self.frame += 1
        return masks, stages, margins
