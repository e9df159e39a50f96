"""FP64 reference of the learned warm-start network, composed from the C
layer oracle (conv_oracle.c).  TEST INFRASTRUCTURE ONLY.

Architecture (channels-last, in_n^3 input):
  enc L1 conv(16->16) conv(16->16), pool; L2 conv(16->32) conv(32->32), pool;
  L3 conv(32->64) conv(64->64), pool; L4 conv(64->128) conv(128->128);
  dec L3 up(L4)++L3 conv(192->64) conv(64->64); L2 up++L2 conv(96->32)
  conv(32->32); L1 up++L1 conv(48->16) conv(16->16); head 1x1x1 16->3.
Every 3x3x3 conv is followed by LeakyReLU(slope).  The input carries m0, m1
in channels 0 and 1 of 16.  Parameter vector: per conv w[27][Ci][Co] then
b[Co]; head w[16][3] then b[3].

With bf16=True every tensor that the device stores in BF16 (inputs,
activations, activation gradients, the convolution weights used by the
matrix cores) is rounded to BF16 (nearest even) at the same place, so the
device kernels are compared against this reference fed the same rounded
operands; with bf16=False it is the plain FP64 network.
"""
import numpy as np

from . import conv3, conv3_t, conv3_dw, lrelu, pool2, up2cat, head

CONVS = [(16, 16, 0), (16, 16, 0), (16, 32, 1), (32, 32, 1), (32, 64, 2), (64, 64, 2), (64, 128, 3),
         (128, 128, 3), (192, 64, 2), (64, 64, 2), (96, 32, 1), (32, 32, 1), (48, 16, 0), (16, 16, 0)]


def layout():
    """Offsets (w, b) of every conv and of the head in the parameter vector."""
    off = 0
    out = []
    for ci, co, _ in CONVS:
        wo = off
        off += 27 * ci * co
        bo = off
        off += co
        out.append((wo, bo))
    hw = off
    off += 48
    hb = off
    off += 3
    return out, hw, hb, off


def bf16_round(x):
    """Round FP64 values to the nearest BF16 (ties to even), returned as FP64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return (u.astype(np.uint32)).view(np.float32).astype(np.float64)


class RefNet:
    def __init__(self, params, slope=0.2, bf16=False):
        self.p = np.asarray(params, dtype=np.float64)
        self.slope = slope
        self.R = bf16_round if bf16 else (lambda a: a)
        self.lay, self.hw, self.hb, self.n = layout()

    def w(self, i):
        ci, co, _ = CONVS[i]
        wo, bo = self.lay[i]
        return self.R(self.p[wo:wo + 27 * ci * co].reshape(27, ci, co)), self.p[bo:bo + co]

    def conv(self, i, x):
        w, b = self.w(i)
        return self.R(lrelu(conv3(x, w, b), self.slope))

    def forward(self, m0, m1):
        R = self.R
        n = m0.shape[0]
        x0 = np.zeros((n, n, n, 16))
        x0[..., 0] = m0
        x0[..., 1] = m1
        t = {"x0": R(x0)}
        t["a1"] = self.conv(0, t["x0"]); t["e1"] = self.conv(1, t["a1"]); t["p1"] = R(pool2(t["e1"]))
        t["a2"] = self.conv(2, t["p1"]); t["e2"] = self.conv(3, t["a2"]); t["p2"] = R(pool2(t["e2"]))
        t["a3"] = self.conv(4, t["p2"]); t["e3"] = self.conv(5, t["a3"]); t["p3"] = R(pool2(t["e3"]))
        t["a4"] = self.conv(6, t["p3"]); t["e4"] = self.conv(7, t["a4"])
        t["c3"] = up2cat(t["e4"], t["e3"]); t["b3"] = self.conv(8, t["c3"]); t["d3"] = self.conv(9, t["b3"])
        t["c2"] = up2cat(t["d3"], t["e2"]); t["b2"] = self.conv(10, t["c2"]); t["d2"] = self.conv(11, t["b2"])
        t["c1"] = up2cat(t["d2"], t["e1"]); t["b1"] = self.conv(12, t["c1"]); t["d1"] = self.conv(13, t["b1"])
        hw = self.p[self.hw:self.hw + 48].reshape(16, 3)
        hb = self.p[self.hb:self.hb + 3]
        v = head(t["d1"], hw, hb)               # (n, n, n, 3)
        self.t = t
        return np.moveaxis(v, -1, 0)            # (3, n, n, n)

    def loss_grad(self, m0, m1, label):
        """0.5 mean (v - label)^2 and its gradient w.r.t. the parameters."""
        R = self.R
        v = self.forward(m0, m1)
        r = v - label
        L = 0.5 * np.mean(r * r)
        gv = np.moveaxis(r / r.size, 0, -1)     # (n, n, n, 3)
        t = self.t
        g = np.zeros(self.n)
        hw = self.p[self.hw:self.hw + 48].reshape(16, 3)
        g[self.hw:self.hw + 48] = np.einsum("zyxi,zyxo->io", t["d1"], gv).ravel()
        g[self.hb:self.hb + 3] = gv.sum(axis=(0, 1, 2))
        gd1 = R(gv @ hw.T)

        def cbwd(i, x_in, y_out, gout, want_gin=True):
            ci, co, _ = CONVS[i]
            wo, bo = self.lay[i]
            dz = R(np.where(y_out > 0, gout, self.slope * gout))
            gw, gb = conv3_dw(x_in, dz)
            g[wo:wo + 27 * ci * co] = gw.ravel()
            g[bo:bo + co] = gb
            if want_gin:
                w, _ = self.w(i)
                return R(conv3_t(dz, w))
            return None

        def up_bwd(gc, ca):
            ga = gc[..., :ca]
            n2 = ga.shape[0] // 2
            ga = ga.reshape(n2, 2, n2, 2, n2, 2, ca).sum(axis=(1, 3, 5))
            return R(ga), gc[..., ca:]

        def pool_bwd(gp, gfine):
            up = np.repeat(np.repeat(np.repeat(gp, 2, 0), 2, 1), 2, 2) / 8.0
            return R(gfine + up)

        gb1 = cbwd(13, t["b1"], t["d1"], gd1)
        gc1 = cbwd(12, t["c1"], t["b1"], gb1)
        gd2, ge1 = up_bwd(gc1, 32)
        gb2 = cbwd(11, t["b2"], t["d2"], gd2)
        gc2 = cbwd(10, t["c2"], t["b2"], gb2)
        gd3, ge2 = up_bwd(gc2, 64)
        gb3 = cbwd(9, t["b3"], t["d3"], gd3)
        gc3 = cbwd(8, t["c3"], t["b3"], gb3)
        ge4, ge3 = up_bwd(gc3, 128)
        ga4 = cbwd(7, t["a4"], t["e4"], ge4)
        gp3 = cbwd(6, t["p3"], t["a4"], ga4)
        ge3 = pool_bwd(gp3, ge3)
        ga3 = cbwd(5, t["a3"], t["e3"], ge3)
        gp2 = cbwd(4, t["p2"], t["a3"], ga3)
        ge2 = pool_bwd(gp2, ge2)
        ga2 = cbwd(3, t["a2"], t["e2"], ge2)
        gp1 = cbwd(2, t["p1"], t["a2"], ga2)
        ge1 = pool_bwd(gp1, ge1)
        ga1 = cbwd(1, t["a1"], t["e1"], ge1)
        cbwd(0, t["x0"], t["a1"], ga1, want_gin=False)
        return L, g


def init_params(seed, scale_head=0.0):
    """Seeded He-uniform convolution weights, zero biases; head weights
    N(0, scale_head^2) (zero by default)."""
    rng = np.random.default_rng(seed)
    lay, hw, hb, n = layout()
    p = np.zeros(n)
    for (ci, co, _), (wo, bo) in zip(CONVS, lay):
        a = np.sqrt(6.0 / (27 * ci))
        p[wo:wo + 27 * ci * co] = rng.uniform(-a, a, 27 * ci * co)
    p[hw:hw + 48] = scale_head * rng.standard_normal(48)
    return p
