"""The paper's detector input on the GPU: the U-Net on summary-image patches
(include/seg_nn.h, seg_nn_st_*; Sec. III-C).

Bars:
- patches bit-exact against the reference;
- the weighted merge within 1e-6 (the GPU accumulates in FP64 and rounds to
  FP32);
- loss, gradients and probabilities against the FP64 reference at the same
  BF16 weights in its BF16 numerics mode (every product rounds its operands
  to BF16, tensors are stored in FP32, as in the kernels): every layer's
  gradient within 2e-2 norm-wise, on every convolution path;
- the session's probability maps bit-identical to the network run on the
  session's own S and T;
- after training on simulated summary pairs, segmentation of held-out
  recordings against their planted truth.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import nn_ref, unet_st
from paper_2403_16438_amd import Session, abi, segment_video, to_device_frames
from paper_2403_16438_amd.unet import SummaryUNet, he_init, merge, param_layout, patch_count, patches
from synth import preset, simulate

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def test_layout_matches_reference():
    lay = param_layout()
    assert [(n, r, c) for n, r, c, _, _ in lay] == [(n, r, c) for n, r, c in unet_st.LAYERS]
    at = 0
    for name, r, c, wo, bo in lay:
        assert wo == at and bo == at + r * c
        at += r * c + nn_ref.bias_len(name, r)
    assert at == unet_st.n_params()


@pytest.mark.parametrize("H,W", [(64, 64), (100, 150), (256, 256), (67, 130)])
def test_patches_and_merge(H, W):
    rng = np.random.default_rng(H * W)
    S = rng.uniform(500, 1500, (H, W)).astype(np.float32)
    T = rng.uniform(0, 80, (H, W)).astype(np.float32)
    p = patches(torch.from_numpy(S).to(DEV), torch.from_numpy(T).to(DEV)).cpu().numpy()
    assert patch_count(H, W) == p.shape[0]
    assert np.array_equal(p, unet_st.patches(S, T).astype(np.float32))
    prob = rng.random((p.shape[0], 64, 64)).astype(np.float32)
    got = merge(torch.from_numpy(prob).to(DEV), H, W).cpu().numpy()
    ref = unet_st.merge(prob.astype(np.float64), H, W)
    assert np.abs(got - ref).max() <= 1e-6


@pytest.fixture(scope="module")
def case():
    rng = np.random.default_rng(12)
    S = rng.uniform(800, 1200, (2, 16, 16))
    T = rng.uniform(0, 60, (2, 16, 16))
    T[0, 4:8, 5:9] += 200
    T[1, 9:13, 2:6] += 150
    st = np.stack([S, T], axis=1).astype(np.float32)
    labels = np.zeros((2, 16, 16), np.float32)
    labels[0, 4:8, 5:9] = 1
    labels[1, 9:13, 2:6] = 1
    theta = he_init(3)
    theta += (0.01 * rng.standard_normal(theta.size)).astype(np.float32)
    return st, labels, theta


BF16 = nn_ref.Numerics(bf16=True)


def _per_layer(g, rg):
    errs, cos = {}, {}
    for name, r, c, wo, bo in param_layout():
        sl = slice(wo, bo + nn_ref.bias_len(name, r))
        den = np.linalg.norm(rg[sl])
        errs[name] = np.linalg.norm(g[sl] - rg[sl]) / max(den, 1e-30)
        cos[name] = float(g[sl] @ rg[sl] / max(np.linalg.norm(g[sl]) * den, 1e-30))
    return errs, cos


def _ref_theta(theta):
    t = theta.astype(np.float64).copy()
    for name, r, c, wo, bo in param_layout():
        t[wo:wo + r * c] = nn_ref.bf16_round(theta[wo:wo + r * c])
    return t


def test_loss_and_gradients_vs_reference(case):
    st, labels, theta = case
    net = SummaryUNet(2, 16, 16, theta)
    loss, g = net.backward(torch.from_numpy(st).to(DEV), torch.from_numpy(labels).to(DEV), want_grad=True)
    g = g.cpu().numpy().astype(np.float64)
    rloss, rg = unet_st.loss_and_grad(_ref_theta(theta), st.astype(np.float64), labels, BF16)
    errs, cos = _per_layer(g, rg)
    print("loss", loss, "reference", rloss)
    print("norm-wise gradient error per layer (BF16 reference):", {k: f"{v:.1e}" for k, v in errs.items()})
    assert max(errs.values()) <= 2e-2, errs
    assert min(cos.values()) >= 0.999, cos
    assert abs(loss - rloss) <= 2e-3 * abs(rloss), (loss, rloss)


def test_forward_probabilities(case):
    st, labels, theta = case
    net = SummaryUNet(2, 16, 16, theta)
    p = net.forward(torch.from_numpy(st).to(DEV)).cpu().numpy()
    logit, _, _ = unet_st.forward(_ref_theta(theta), st.astype(np.float64), BF16)
    err = np.abs(p - 1.0 / (1.0 + np.exp(-logit)))
    print("prob error max", err.max(), "mean", err.mean())
    assert err.mean() <= 2e-3 and err.max() <= 2e-2


@pytest.mark.parametrize("B,H,W", [(1, 24, 24), (2, 24, 40), (2, 32, 16)])
def test_convolution_paths_vs_reference(B, H, W):
    """Shapes that route the convolutions through every kernel path: the
    direct halo kernel (W a multiple of 8 whose column block divides the
    tile), the product that gathers the im2col itself (W = 24 or 40 at full
    resolution), im2col + product (W = 12, 10, 6 or 4 at lower resolutions),
    and the transposed convolutions both fused (B H W / 16 a multiple of 8)
    and through the product + scatter (B = 1, 24 x 24)."""
    rng = np.random.default_rng(B * 1000 + H * W)
    S = rng.uniform(800, 1200, (B, H, W))
    T = rng.uniform(0, 60, (B, H, W))
    T[:, 4:9, 5:10] += 180
    st = np.stack([S, T], axis=1).astype(np.float32)
    labels = np.zeros((B, H, W), np.float32)
    labels[:, 4:9, 5:10] = 1
    theta = he_init(5)
    theta += (0.01 * rng.standard_normal(theta.size)).astype(np.float32)
    net = SummaryUNet(B, H, W, theta)
    sd = torch.from_numpy(st).to(DEV)
    p = net.forward(sd).cpu().numpy()
    rt = _ref_theta(theta)
    # against the reference in its BF16 numerics mode (operands of every
    # product rounded to BF16, tensors stored in FP32, as the kernels do)
    logit, _, _ = unet_st.forward(rt, st.astype(np.float64), BF16)
    err = np.abs(p - 1.0 / (1.0 + np.exp(-logit)))
    print("prob error max", err.max(), "mean", err.mean(), "logit range", logit.min(), logit.max())
    loss, g = net.backward(sd, torch.from_numpy(labels).to(DEV), want_grad=True)
    g = g.cpu().numpy().astype(np.float64)
    rloss, rg = unet_st.loss_and_grad(rt, st.astype(np.float64), labels, BF16)
    errs, cos = _per_layer(g, rg)
    print("loss", loss, "reference", rloss)
    print("norm-wise gradient error per layer (BF16 reference):", {k: f"{v:.1e}" for k, v in errs.items()})
    # what remains are BF16 roundings that FP32 accumulation (GPU) and FP64
    # sums (reference) put on either side of a rounding boundary; an indexing
    # or padding mistake moves many pixels by 0.1 or more
    assert err.mean() <= 2e-3 and err.max() <= 3e-2
    assert max(errs.values()) <= 2e-2, errs
    assert min(cos.values()) >= 0.999, cos
    assert abs(loss - rloss) <= 2e-3 * abs(rloss), (loss, rloss)
    net.close()


@pytest.mark.parametrize("B,H,W", [(4, 64, 64), (2, 68, 320)])
def test_bf16_activation_forward_equals_training_forward(B, H, W):
    """The forward-only call keeps the activations as BF16 in channel blocks
    where every layer fits the BF16 kernels (H a multiple of 4, W of 64), with
    the poolings and the output layer in convolution epilogues; every
    consumer rounds its input to BF16 anyway and every product sums in the
    same order, so its logits must equal, bit for bit, those of the training
    forward (FP32 activations) that the backward call runs. 68 x 320 leaves
    ragged tiles at every level (rows 17 at the lowest, columns 160 and 80)."""
    rng = np.random.default_rng(11)
    S = rng.uniform(800, 1200, (B, H, W))
    T = rng.uniform(0, 60, (B, H, W))
    T[:, 20:28, 30:38] += 180
    st = torch.from_numpy(np.stack([S, T], axis=1).astype(np.float32)).to(DEV)
    labels = torch.zeros((B, H, W), dtype=torch.float32, device=DEV)
    labels[:, 20:28, 30:38] = 1
    theta = he_init(3)
    theta += (0.01 * rng.standard_normal(theta.size)).astype(np.float32)
    net = SummaryUNet(B, H, W, theta)
    p = net.forward(st)
    li = net.logits().clone()
    net.backward(st, labels)
    lt = net.logits()
    torch.cuda.synchronize()
    assert torch.equal(li, lt), (li - lt).abs().max().item()
    assert torch.equal(p, torch.sigmoid(lt)) or (p - torch.sigmoid(lt)).abs().max().item() < 1e-6
    net.close()


def test_rmsprop_reduces_loss(case):
    st, labels, theta = case
    net = SummaryUNet(2, 16, 16, theta)
    sd, ld = torch.from_numpy(st).to(DEV), torch.from_numpy(labels).to(DEV)
    losses = []
    for _ in range(40):
        loss, _ = net.backward(sd, ld)
        losses.append(loss)
        net.step(lr=1e-3)
    assert losses[-1] < 0.5 * losses[0], losses[::8]


def test_models_and_errors():
    net = SummaryUNet(4, 64, 64)
    frames_net_sess = Session(64, 64, 100, detector=abi.SEG_DET_SURROGATE)
    with pytest.raises(abi.SegError) as e:
        frames_net_sess.set_model(net)                 # a summary network on the frame detector
    assert e.value.code == abi.SEG_E_SHAPE
    s = Session(128, 128, 100, detector=abi.SEG_DET_UNET, event_z=0.5, min_event_segs=2)
    d = torch.zeros((100, 128, 128), dtype=torch.int16, device=DEV)
    with pytest.raises(abi.SegError) as e:
        s.push(d)
    assert e.value.code == abi.SEG_E_NOMODEL
    small = SummaryUNet(4, 32, 32)
    with pytest.raises(abi.SegError) as e:
        s.set_model(small)                             # patches must be 64 x 64
    assert e.value.code == abi.SEG_E_SHAPE
    with pytest.raises(abi.SegError):
        Session(48, 128, 100, detector=abi.SEG_DET_UNET)
    st = torch.zeros((1, 2, 64, 64), dtype=torch.float32, device=DEV)
    with pytest.raises(abi.SegError) as e:
        abi.check(abi.lib.seg_nn_forward(net.handle, abi.C.c_void_p(st.data_ptr()), 1, None, None), "fwd")
    assert e.value.code == abi.SEG_E_STATE


@pytest.fixture(scope="module")
def trained():
    from paper_2403_16438_amd.train import SummaryBank, train_unet
    bank = SummaryBank(120, device="cuda")
    net, losses = train_unet(steps=5000, batch=32, lr=1e-3, bank=bank)
    return net, losses


def test_training_converges(trained):
    net, losses = trained
    first, last = np.mean(losses[:50]), np.mean(losses[-200:])
    print("summary U-Net loss", first, "->", last)
    assert last < 0.5 * first


def test_session_maps_equal_network(trained):
    """The session's probability maps are the network's merged output on the
    session's own S and T, bit for bit."""
    net, _ = trained
    video, _ = simulate(preset(4, height=128, width=128, frames=500, n_neurons=6, n_overlap=1), 77)
    sess = segment_video(video, net=net)
    S = sess.segment_maps(abi.SEG_MAP_S)
    T = sess.segment_maps(abi.SEG_MAP_T)
    P = sess.segment_maps(abi.SEG_MAP_P)
    for i in (0, 4, 9):
        assert torch.equal(P[i], net.segment_map(S[i].contiguous(), T[i].contiguous())), i


def test_segmentation_quality(trained, record_property):
    """Held-out recordings of the training kind: planted-truth F1 of the
    paper's detector beside the plain one. The detector's event threshold
    (0.7) and c_min (3) were chosen on other seeds (81-84) of the same kind;
    the paper's OR aggregation (c_min = 1) is recorded beside them."""
    net, _ = trained
    f_unet, f_or, f_plain = [], [], []
    for seed in (91, 92, 93):
        video, truth = simulate(preset(4, height=128, width=128, frames=1000, n_neurons=8, n_overlap=2,
                                       edge_margin=10.0), seed)
        f_unet.append(oracle.match_f1(segment_video(video, net=net).footprints()["masks"], truth.masks())["f1"])
        f_or.append(oracle.match_f1(segment_video(video, net=net, min_event_segs=1).footprints()["masks"],
                                    truth.masks())["f1"])
        f_plain.append(oracle.match_f1(segment_video(video).footprints()["masks"], truth.masks())["f1"])
    record_property("f1_unet", float(np.mean(f_unet)))
    record_property("f1_unet_or", float(np.mean(f_or)))
    record_property("f1_plain", float(np.mean(f_plain)))
    print("F1 summary U-Net", f_unet, "with c_min = 1", f_or, "plain", f_plain)
    assert np.mean(f_unet) >= 0.85      # measured 0.906 (c_min = 1: 0.873, plain 0.96)
