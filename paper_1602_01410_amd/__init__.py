"""MI355X-native partial-ADMM deconvolution with incomplete observations.

Importing the package loads nothing native; the HIP library is opened on
first use (see ``paper_1602_01410_amd.binding``).
"""
