"""The paper's printed constants (tests/golden/paper_constants.json) are the
defaults the oracle and the library use."""
import json
import os

import numpy as np

import oracle as O

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def test_training_defaults_follow_the_paper():
    import inspect
    sig = inspect.signature(O.nif_train_step)
    assert sig.parameters["delta"].default == GOLD["huber_delta"]["value"]
    assert sig.parameters["lr"].default == GOLD["adam_learning_rate"]["value"]


def test_roulette_start_default_follows_the_paper():
    import inspect
    assert inspect.signature(O.render_desc).parameters["rr_start"].default == \
        GOLD["roulette_start_depth"]["value"]


def test_paper_nif_size_is_consistent_with_fp16_weights():
    # the paper's network is 97 KiB of FP16 weights (Fig. 1 and Table 2
    # captions, "H128, L5"): 40-d features, four dense-ReLU layers of 128
    # with the second narrowed to 128 - 40 so that the features concatenated
    # to its output make 128 inputs, and the linear output layer -- five
    # trainable layers.  Five dense-ReLU layers would be a third larger.
    kib = GOLD["nif_size_kib_h128_l5"]["value"]
    paper = O.nif_param_count(O.nif_shape(10, 128, 4, O.COLOUR_YUV, 2)) * 2 / 1024
    assert abs(paper - kib) / kib < 0.01
    five = O.nif_param_count(O.nif_shape(10, 128, 5, O.COLOUR_YUV, 2)) * 2 / 1024
    assert five > 1.3 * kib
    # the plain 64-d / H96 / L5 network of the workload is 43,779 parameters
    # = 85.5 KiB in FP16, the same order
    n = O.nif_param_count(O.nif_shape(16, 96, 5))
    assert abs(n * 2 / 1024 - 85.5) < 0.1
    assert n * 2 / 1024 < kib


def test_fp16_extent_node_saving():
    # 32 B -> 24 B nodes is the 25 % saving the paper reports
    a, b = GOLD["bvh_node_bytes_fp32"]["value"], GOLD["bvh_node_bytes_fp16_extent"]["value"]
    assert np.isclose(1 - b / a, 0.25)
