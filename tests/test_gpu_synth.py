"""The GPU evaluation of the synthetic streams gives the same bytes as frames.py."""
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fast():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from synth import fast
    return fast


def test_fast_generator_matches_definition(fast):
    from synth import frames as F
    specs = [F.cfg0().streams[0], F.cfg1(n_test=3).streams[0]]
    specs += F.mixed_streams(6, seed=9, n_test=4)[0]
    specs.append(F.StreamSpec(100, 37, 2, 3, seed=4, fg="ellipses", fg_coverage=0.2, drift_amp=0.3, bimodal_frac=0.5))
    # widths that end in a partial 16-pixel group, and narrower than one group
    for W, H in [(33, 17), (7, 5), (16, 3), (47, 2), (1, 1)]:
        specs.append(F.StreamSpec(W, H, 2, 3, seed=6, fg="ellipses", fg_coverage=0.3, drift_amp=0.2,
                                  bimodal_frac=0.3, block=5))
    specs.append(F.StreamSpec(70, 20, 2, 3, seed=7, fg="rect", rect_size=9))
    for spec in specs:
        ids = [0, 1, spec.n_train, spec.n_frames - 1]
        print(f"[case] {spec.width}x{spec.height} frames {ids}", flush=True)
        want = F.make_frames(spec, ids, device="cuda")
        got = torch.zeros_like(want)
        fast.make_frames_gpu(spec, ids, got)
        torch.cuda.synchronize()
        W = spec.width
        assert torch.equal(got[:, :, : 3 * W], want[:, :, : 3 * W]), (spec.width, spec.height)
