"""Convolutional subspace predictor binding (filled in with the CNN kernels)."""


class Cnn:
    pass
