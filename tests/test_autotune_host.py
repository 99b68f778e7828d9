"""Host-side checks of the autotuner's cache keys and candidate limits."""
import inputs


def test_autotune_key_separates_receiver_slab_heights():
    from paper_2203_16573_amd import autotune
    wl = inputs.workload(2)
    k0 = autotune.shape_key(wl.prob, 1, "f32")
    k5 = autotune.shape_key(wl.prob.replace(rslab_dz=-5), 1, "f32")
    k40 = autotune.shape_key(wl.prob.replace(rslab_dz=-40), 1, "f32")
    assert len({k0, k5, k40}) == 3
    # a receiver-side slab too tall for the multi-step slab kernel keeps the
    # tuner off that kernel
    assert autotune.tallest_slab(wl.prob) <= autotune.SLAB_MAXZ
    assert autotune.tallest_slab(wl.prob.replace(rslab_dz=-40)) > autotune.SLAB_MAXZ
