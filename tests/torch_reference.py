"""Second, independent float64 evaluation of the network on the CPU, built
from torch.nn.functional library routines (conv2d, conv_transpose2d,
interpolate, grid_sample). Used only to cross-check the numpy oracle on
random weights, where the paper fixes no output values; it shares no code
with the oracle and takes its weights straight from the generator's arrays,
not from the weights file.
"""
import torch
import torch.nn.functional as Fn


def _t(a):
    return torch.as_tensor(a, dtype=torch.float64)


def _conv(Wd, name, x, stride, act=True):
    w, b = Wd[name]
    y = Fn.conv2d(x, _t(w), _t(b), stride=stride, padding=1)
    return torch.relu(y) if act else y


def _convT(Wd, name, x, act=True):
    w, b = Wd[name]
    y = Fn.conv_transpose2d(x, _t(w), _t(b), stride=2, padding=1)
    return torch.relu(y) if act else y


def _resize(x, h, w):
    return Fn.interpolate(x, size=(h, w), mode="bilinear", align_corners=False)


def _warp(img, flow):
    n, c, h, w = img.shape
    ys = torch.arange(h, dtype=torch.float64).view(1, h, 1).expand(n, h, w)
    xs = torch.arange(w, dtype=torch.float64).view(1, 1, w).expand(n, h, w)
    gx = 2.0 * (xs + flow[:, 0]) / (w - 1) - 1.0
    gy = 2.0 * (ys + flow[:, 1]) / (h - 1) - 1.0
    grid = torch.stack([gx, gy], dim=-1)
    return Fn.grid_sample(img, grid, mode="bilinear", padding_mode="border", align_corners=True)


def _vib(Wd, s, x):
    a = _conv(Wd, f"vib{s}.conv1", x, 2)
    a = _conv(Wd, f"vib{s}.conv2", a, 2)
    for i in range(3, 9):
        a = _conv(Wd, f"vib{s}.conv{i}", a, 1)
    a = _convT(Wd, f"vib{s}.convT1", a)
    return _convT(Wd, f"vib{s}.convT2", a, act=False)


def forward(xl, xr, t, Wd, t_plane=True):
    xl = _t(xl)[None]
    xr = _t(xr)[None]
    H, W = xl.shape[-2:]
    Hp, Wp = (H + 15) // 16 * 16, (W + 15) // 16 * 16
    Xl = Fn.pad(xl, (0, Wp - W, 0, Hp - H), mode="replicate")
    Xr = Fn.pad(xr, (0, Wp - W, 0, Hp - H), mode="replicate")
    flow = mask = None
    for s in range(3):
        h, w = Hp // 4 * 2 ** s, Wp // 4 * 2 ** s
        L = Xl if s == 2 else _resize(Xl, h, w)
        R = Xr if s == 2 else _resize(Xr, h, w)
        extra = [torch.full((1, 1, h, w), float(t), dtype=torch.float64)] if t_plane else []
        if s == 0:
            out = _vib(Wd, 0, torch.cat([L, R] + extra, 1))
            flow, mask = out[:, :4], out[:, 4:]
        else:
            fu = _resize(flow, h, w) * 2.0
            mu = _resize(mask, h, w)
            inp = torch.cat([L, R, _warp(L, fu[:, :2]), _warp(R, fu[:, 2:]), mu, fu] + extra, 1)
            out = _vib(Wd, s, inp)
            flow, mask = fu + out[:, :4], mu + out[:, 4:]
    wl = _warp(Xl, flow[:, :2])
    wr = _warp(Xr, flow[:, 2:])
    m = torch.sigmoid(mask)
    blended = m * wl + (1 - m) * wr

    def ctx(x):
        feats = []
        for k in range(4):
            x = _conv(Wd, f"ctx.conv{2 * k + 1}", x, 2)
            x = _conv(Wd, f"ctx.conv{2 * k + 2}", x, 1)
            feats.append(x)
        return feats

    fl, fr = ctx(Xl), ctx(Xr)
    warped = []
    fk = flow
    for k in range(4):
        fk = Fn.avg_pool2d(fk, 2) * 0.5
        warped.append(torch.cat([_warp(fl[k], fk[:, :2]), _warp(fr[k], fk[:, 2:])], 1))

    def enc(k, z):
        z = _conv(Wd, f"unet.enc{2 * k + 1}", z, 2)
        return _conv(Wd, f"unet.enc{2 * k + 2}", z, 1)

    e1 = enc(0, torch.cat([Xl, Xr, wl, wr, mask, flow], 1))
    e2 = enc(1, torch.cat([e1, warped[0]], 1))
    e3 = enc(2, torch.cat([e2, warped[1]], 1))
    e4 = enc(3, torch.cat([e3, warped[2]], 1))
    y = _convT(Wd, "unet.dec1", torch.cat([e4, warped[3]], 1))
    y = _convT(Wd, "unet.dec2", torch.cat([y, e3], 1))
    y = _convT(Wd, "unet.dec3", torch.cat([y, e2], 1))
    y = _convT(Wd, "unet.dec4", torch.cat([y, e1], 1))
    r = torch.sigmoid(_conv(Wd, "unet.head", y, 1, act=False))
    res = torch.clamp(blended + 2 * r - 1, 0.0, 1.0)
    return res[0, :, :H, :W].numpy()
